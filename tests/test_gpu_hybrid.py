"""Dynamic CPU/GPU scheduling (Sec. 3.3) of Lennard-Jones cell-pair requests: each step splits the
task queue by the running per-item times, runs the front on the CPU kernel and the rest as one
combined GPU launch, and the two parts must add up to the oracle's forces."""
import time

import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from test_hybrid import lj_task_records

pytestmark = pytest.mark.gpu


def test_hybrid_steps_split_by_measured_ratio():
    import torch
    print("[gpu] hybrid CPU/GPU LJ steps, FCC 11000", flush=True)
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=92)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 10), L, 2.5, **W.LJ_TWO_TYPES)
    ref = O.lj_tasks(w)
    items = np.where(w.self_flag != 0, w.i_count, w.i_count + w.j_count).astype(np.int64)
    ctx = gc.Context(0)
    src = torch.from_numpy(np.ascontiguousarray(w.rec)).cuda()
    eps, sig, mass = (torch.from_numpy(x).cuda() for x in (w.eps_t, w.sig_t, w.mass_t))
    pool = gc.Pool(ctx, w.n, w.n)
    pool.set_source(src)
    prm = gc.lj_params(eps, sig, mass, w.rcut)
    acc_dev = torch.zeros((w.n, 4), dtype=torch.float32, device="cuda")
    # one launch over every task first: kernel loading stays out of the timings
    t, r = lj_task_records(w)
    b = gc.Batch(ctx, gc.KIND_LJ, w.n)
    b.submit(t, r)
    b.commit()
    b.reorganize(pool, gc.REORG_NONE)
    b.launch(prm, None, acc_dev)
    torch.cuda.synchronize()
    b.destroy()
    h = gc.Hybrid()
    for step in range(4):
        st = h.state()
        k, kc = h.split(items)
        # the rule: the CPU's share of the items is tau_gpu / (tau_cpu + tau_gpu) (one half untimed),
        # reached at the k-th request
        share = 0.5 if step == 0 else st["tau_gpu"] / (st["tau_cpu"] + st["tau_gpu"])
        want = share * items.sum()
        cum = np.cumsum(items)
        assert (k == 0 and want <= 0) or (cum[k - 1] >= want and (k == 1 or cum[k - 2] < want))
        acc = np.zeros((w.n, 4), np.float32)
        acc_dev.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b = None
        if k < w.n_tasks:  # the GPU part goes out first and runs while the CPU computes its part
            t, r = lj_task_records(w, np.arange(k, w.n_tasks))
            b = gc.Batch(ctx, gc.KIND_LJ, w.n)
            b.submit(t, r)
            b.commit()
            e0.record()
            b.reorganize(pool, gc.REORG_NONE)
            b.launch(prm, None, acc_dev)
            e1.record()
        if k > 0:
            t, r = lj_task_records(w, np.arange(k))
            tc0 = time.perf_counter()
            gc.lj_forces_cpu(t, r, w.rec, w.eps_t, w.sig_t, w.mass_t, w.rcut, acc)
            h.record(gc.DEVICE_CPU, int(kc), time.perf_counter() - tc0)
        if b is not None:
            e1.synchronize()
            h.record(gc.DEVICE_GPU, int(items[k:].sum()), e0.elapsed_time(e1) * 1e-3)
            b.destroy()
        total = acc[:, :3].astype(np.float64) + acc_dev.cpu().numpy()[:, :3].astype(np.float64)
        nc = np.diff(w.cell_start)
        keep = nc > 0
        err = O.per_task_rel_l2(total, ref, w.cell_start[:-1][keep], nc[keep], floor_frac=1e-3)
        st = h.state()
        print(f"[gpu] step {step}: {k} of {w.n_tasks} requests on the CPU, tau cpu {st['tau_cpu']:.2e} "
              f"gpu {st['tau_gpu']:.2e} s/item, max cell rel L2 {err.max():.2e}", flush=True)
        assert err.max() <= 1e-5, (step, err.max())
    s = h.state()
    assert s["runs_cpu"] >= 1 and s["runs_gpu"] >= 1
    h.destroy()
    pool.destroy()
    ctx.close()
