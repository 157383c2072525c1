"""Dynamic CPU/GPU scheduling (Sec. 3.3) through the C-ABI: the split rule on hand-worked cases,
and the CPU Lennard-Jones kernel against the FP64 oracle (host code, no GPU)."""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W


def test_half_split_until_both_devices_are_timed():
    h = gc.Hybrid()
    assert h.split([10, 10, 10, 10]) == (2, 20)    # share 1/2: 20 items, reached at the second request
    h.record(gc.DEVICE_CPU, 10, 30.0)
    assert h.split([10, 10, 10, 10]) == (2, 20)    # the GPU has no record yet
    h.destroy()


def test_share_follows_the_running_means():
    h = gc.Hybrid()
    h.record(gc.DEVICE_CPU, 10, 30.0)     # 3 s per item
    h.record(gc.DEVICE_CPU, 5, 20.0)      # 4 s per item: mean 3.5
    h.record(gc.DEVICE_GPU, 100, 50.0)    # 0.5 s per item
    s = h.state()
    assert (s["tau_cpu"], s["tau_gpu"], s["runs_cpu"], s["runs_gpu"]) == (3.5, 0.5, 2, 1)
    # CPU share 0.5 / (3.5 + 0.5) = 1/8 of 80 items = 10: reached at the first request
    assert h.split([10] * 8) == (1, 10)
    # 1/8 of 160 = 20: the running sum 15, 30 reaches it at the second request (which goes to the CPU)
    assert h.split([15, 15, 50, 80]) == (2, 30)
    h.destroy()


def test_uneven_requests_are_counted_by_their_items():
    h = gc.Hybrid()
    assert h.split([100, 1, 1, 1, 100]) == (3, 102)  # half of 203 is 101.5
    assert h.split([]) == (0, 0)
    h.destroy()


def test_an_instant_gpu_takes_everything():
    h = gc.Hybrid()
    h.record(gc.DEVICE_CPU, 10, 1.0)
    h.record(gc.DEVICE_GPU, 10, 0.0)
    assert h.split([5, 5, 5]) == (0, 0)
    h.destroy()


def test_invalid_records_leave_the_state_unchanged():
    h = gc.Hybrid()
    for dev, items, sec in ((2, 10, 1.0), (gc.DEVICE_CPU, 0, 1.0), (gc.DEVICE_GPU, 5, -1.0)):
        with pytest.raises(gc.GcError):
            h.record(dev, items, sec)
    with pytest.raises(gc.GcError):
        h.split([3, -1])
    assert h.state() == {"tau_cpu": 0.0, "tau_gpu": 0.0, "runs_cpu": 0, "runs_gpu": 0}
    h.destroy()


def lj_task_records(w, sel=None):
    sel = np.arange(w.n_tasks) if sel is None else sel
    t = gc.tasks_from_csr(w.i_begin[sel], w.i_count[sel], np.arange(sel.size, dtype=np.int32),
                          np.ones(sel.size, np.int32), flags=np.where(w.self_flag[sel] != 0, gc.TASK_SELF, 0),
                          shift=w.shift[sel])
    r = np.stack([w.j_begin[sel], w.j_count[sel]], axis=1).astype(np.int32)
    return t, r


def test_cpu_kernel_matches_oracle_and_splits_add_up():
    xyz, v, L = W.fcc_modulated(8, 7, 7, 0.8442, 1500, seed=91)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 9), L, 2.5, **W.LJ_TWO_TYPES)
    t, r = lj_task_records(w)
    acc = np.zeros((w.n, 4), np.float32)
    gc.lj_forces_cpu(t, r, w.rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, acc, n_threads=3)
    ref = O.lj_tasks(w)
    nc = np.diff(w.cell_start)
    keep = nc > 0
    err = O.per_task_rel_l2(acc[:, :3].astype(np.float64), ref, w.cell_start[:-1][keep], nc[keep], floor_frac=1e-3)
    assert err.max() <= 1e-5, err.max()
    assert np.all(acc[:, 3] == 0.0)
    # two halves of the task list add up to the whole
    k = w.n_tasks // 3
    a1 = np.zeros_like(acc)
    t1, r1 = lj_task_records(w, np.arange(k))
    t2, r2 = lj_task_records(w, np.arange(k, w.n_tasks))
    gc.lj_forces_cpu(t1, r1, w.rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, a1)
    gc.lj_forces_cpu(t2, r2, w.rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, a1)
    assert np.abs(a1 - acc).max() <= 1e-5 * np.abs(acc).max()


def test_cpu_kernel_rejects_bad_input():
    w = W.lj_small()
    t, r = lj_task_records(w)
    acc = np.zeros((w.n, 4), np.float32)
    rec = w.rec.copy()
    rec[3, 3] = 7.0  # a type outside [0, n_types)
    with pytest.raises(gc.GcError):
        gc.lj_forces_cpu(t, r, rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, acc)
    r2 = r.copy()
    r2[0, 1] = w.n  # a range past the ids
    with pytest.raises(gc.GcError):
        gc.lj_forces_cpu(t, r2, w.rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, acc)
    assert np.all(acc == 0.0)
