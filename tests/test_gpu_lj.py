"""GPU parity of the combined Lennard-Jones kernel (cell-pair tasks) against the FP64 oracle.

Bar: per-cell relative L2 <= 1e-5 of the accelerations (cells with a near-zero reference force are
measured against 1e-3 x the median cell norm).  The cutoff decision is taken in FP32 on both sides.
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def lj_tasks(w):
    ranges = np.stack([w.j_begin, w.j_count], axis=1).astype(np.int32)
    t = gc.tasks_from_csr(w.i_begin, w.i_count, np.arange(w.n_tasks, dtype=np.int32), np.ones(w.n_tasks, np.int32),
                          flags=np.where(w.self_flag != 0, gc.TASK_SELF, 0), shift=w.shift)
    return t, ranges


class LJRig:
    def __init__(self, ctx, w):
        import torch
        self.torch, self.ctx, self.w = torch, ctx, w
        self.src = torch.from_numpy(np.ascontiguousarray(w.rec)).cuda()
        self.eps = torch.from_numpy(w.eps_t).cuda()
        self.sig = torch.from_numpy(w.sig_t).cuda()
        self.mass = torch.from_numpy(w.mass_t).cuda()
        self.acc = torch.zeros((w.n, 4), dtype=torch.float32, device="cuda")
        self.pool = gc.Pool(ctx, w.n, w.n)
        self.pool.set_source(self.src)
        t, r = lj_tasks(w)
        self.b = gc.Batch(ctx, gc.KIND_LJ, w.n)
        self.b.submit(t, r)
        self.b.commit()

    def run(self, mode, schedule=0):
        self.acc.fill_(np.nan)
        self.b.reorganize(self.pool, mode)
        self.b.launch(gc.lj_params(self.eps, self.sig, self.mass, self.w.rcut, schedule=schedule), None, self.acc)
        self.torch.cuda.synchronize()
        return self.acc.cpu().numpy()

    def close(self):
        self.b.destroy()
        self.pool.destroy()


def per_cell(acc, ref, w, floor=1e-3):
    nc = np.diff(w.cell_start)
    keep = nc > 0
    return O.per_task_rel_l2(acc[:, :3].astype(np.float64), ref, w.cell_start[:-1][keep], nc[keep], floor_frac=floor)


@pytest.mark.parametrize("mode", [gc.REORG_NONE, gc.REORG_PACK, gc.REORG_REDUNDANT])
def test_lj_two_types_small(ctx, mode):
    w = W.lj_small()
    rig = LJRig(ctx, w)
    acc = rig.run(mode)
    ref = O.lj_tasks(w)
    err = per_cell(acc, ref, w, floor=0.0)
    assert err.max() <= TOL, err.max()
    # momentum: sum m a = 0 up to FP32 accumulation
    m = w.mass_t[w.rec[:, 3].astype(int)]
    net = np.sum(m[:, None] * acc[:, :3].astype(np.float64), axis=0)
    assert np.linalg.norm(net) <= 1e-5 * np.sum(m * np.linalg.norm(acc[:, :3], axis=1))
    rig.close()


def test_lj_fcc_modulated_medium_and_persistent(ctx):
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=77)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 5), L, 2.5, **W.LJ_TWO_TYPES)
    rig = LJRig(ctx, w)
    ref = O.lj_tasks(w)
    for sched in (0, 1):
        acc = rig.run(gc.REORG_NONE, schedule=sched)
        err = per_cell(acc, ref, w)
        assert err.max() <= TOL, (sched, err.max())
    rig.close()


def test_lj_cells_of_more_than_64_atoms(ctx):
    # r_c = 5 puts 93 to 165 atoms in a cell: the gather form takes each cell's targets in chunks of
    # 64, each chunk with its own bounding box for the candidate pruning
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=81)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 12), L, 5.0, **W.LJ_TWO_TYPES)
    nc = np.diff(w.cell_start)
    assert nc.max() > 128 and nc[nc > 0].min() > 64
    rig = LJRig(ctx, w)
    ref = O.lj_tasks(w)
    for mode, sched in ((gc.REORG_NONE, 0), (gc.REORG_NONE, 1), (gc.REORG_PACK, 0)):
        acc = rig.run(mode, schedule=sched)
        err = per_cell(acc, ref, w)
        assert err.max() <= TOL, (mode, sched, err.max())
    rig.close()


def test_lj_full_size_one_step(ctx):
    w = W.lj_fcc()
    print(f"[gpu] lj full N={w.n} tasks={w.n_tasks}", flush=True)
    assert w.n == 1048576 and w.n_tasks == 1234800
    rig = LJRig(ctx, w)
    acc = rig.run(gc.REORG_NONE)
    ref = O.lj_tasks(w)
    err = per_cell(acc, ref, w)
    assert err.max() <= TOL, err.max()
    rig.close()


def test_lj_submit_validation(ctx):
    w = W.lj_small()
    b = gc.Batch(ctx, gc.KIND_LJ, w.n)
    t, r = lj_tasks(w)
    t2 = t.copy()
    t2["j_nranges"][0] = 2
    with pytest.raises(gc.GcError) as e:
        b.submit(t2, r)
    assert e.value.status == 1
    t3 = t.copy()
    i = int(np.nonzero(t3["flags"])[0][0])
    t3["i_begin"][i] += 1  # self task whose j range differs from its targets
    t3["i_count"][i] = max(0, t3["i_count"][i] - 1)
    with pytest.raises(gc.GcError):
        b.submit(t3, r)
    assert b.sizes()["tasks"] == 0  # strong guarantee: nothing appended
    b.destroy()


def test_lj_gather_form_is_bitwise_repeatable(ctx):
    # the gather form writes each atom once, without atomics: the same bits on every run, with
    # either schedule, and from the packed records as from the source in place
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=78)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 6), L, 2.5, **W.LJ_TWO_TYPES)
    rig = LJRig(ctx, w)
    runs = [rig.run(gc.REORG_NONE, 0), rig.run(gc.REORG_NONE, 0), rig.run(gc.REORG_NONE, 1), rig.run(gc.REORG_PACK, 0)]
    for r in runs[1:]:
        assert np.array_equal(r.view(np.uint32), runs[0].view(np.uint32))
    err = per_cell(runs[0], O.lj_tasks(w), w)
    assert err.max() <= TOL, err.max()
    rig.close()


def _run_tasks(ctx, w, tasks, mode=gc.REORG_NONE):
    import torch
    src = torch.from_numpy(np.ascontiguousarray(w.rec)).cuda()
    eps, sig, mass = (torch.from_numpy(x).cuda() for x in (w.eps_t, w.sig_t, w.mass_t))
    acc = torch.full((w.n, 4), float("nan"), dtype=torch.float32, device="cuda")
    pool = gc.Pool(ctx, w.n, w.n)
    pool.set_source(src)
    ranges = np.stack([tasks["j_begin"], tasks["j_count"]], axis=1).astype(np.int32)
    n = tasks["i_begin"].shape[0]
    t = gc.tasks_from_csr(tasks["i_begin"], tasks["i_count"], np.arange(n, dtype=np.int32), np.ones(n, np.int32),
                          flags=np.where(tasks["self_flag"] != 0, gc.TASK_SELF, 0), shift=tasks["shift"])
    b = gc.Batch(ctx, gc.KIND_LJ, w.n)
    b.submit(t, ranges)
    b.commit()
    b.reorganize(pool, mode)
    b.launch(gc.lj_params(eps, sig, mass, w.rcut), None, acc)
    torch.cuda.synchronize()
    out = acc.cpu().numpy()
    b.destroy()
    pool.destroy()
    return out


def _task_dict(w, sel=None):
    sel = np.arange(w.n_tasks) if sel is None else sel
    return dict(i_begin=w.i_begin[sel], i_count=w.i_count[sel], j_begin=w.j_begin[sel], j_count=w.j_count[sel],
                self_flag=w.self_flag[sel], shift=w.shift[sel])


def test_lj_partially_overlapping_targets_use_the_atomic_form(ctx):
    # an extra task whose target range straddles two cells: target ranges are no longer equal or
    # disjoint, so the batch runs the half-shell form with atomics; same sums as the oracle's
    w = W.lj_small()
    cs = w.cell_start
    extra = dict(i_begin=np.array([cs[4] + 2], np.int32), i_count=np.array([cs[5] - cs[4]], np.int32),
                 j_begin=np.array([cs[13]], np.int32), j_count=np.array([cs[14] - cs[13]], np.int32),
                 self_flag=np.zeros(1, np.int32), shift=np.zeros((1, 3), np.float32))
    base = _task_dict(w)
    tasks = {k: np.concatenate([base[k], extra[k]]) for k in base}
    acc = _run_tasks(ctx, w, tasks)
    ref = O.lj_tasks(w, tasks=tasks)
    err = per_cell(acc, ref, w, floor=0.0)
    assert err.max() <= TOL, err.max()


def test_lj_gather_form_zeroes_untouched_atoms(ctx):
    # tasks of a few cells only: the gather form writes their targets, every other row is zero
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=79)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 7), L, 2.5, **W.LJ_TWO_TYPES)
    sel = np.nonzero(np.isin(w.i_begin, w.cell_start[[0, 100, 400]]))[0]
    tasks = _task_dict(w, sel)
    acc = _run_tasks(ctx, w, tasks, mode=gc.REORG_PACK)
    ref = O.lj_tasks(w, tasks=tasks)
    touched = np.zeros(w.n, bool)
    for k in range(sel.size):
        touched[tasks["i_begin"][k]:tasks["i_begin"][k] + tasks["i_count"][k]] = True
        touched[tasks["j_begin"][k]:tasks["j_begin"][k] + tasks["j_count"][k]] = True
    assert 0 < touched.sum() < w.n // 2
    assert np.all(acc[~touched] == 0.0)
    # whole cells are touched or not; per touched cell, relative L2 against the oracle
    nc = np.diff(w.cell_start)
    cells = np.nonzero((nc > 0) & touched[np.minimum(w.cell_start[:-1], w.n - 1)])[0]
    err = O.per_task_rel_l2(acc[:, :3].astype(np.float64), ref, w.cell_start[cells], nc[cells], floor_frac=0.0)
    assert err.max() <= TOL, err.max()


def test_lj_in_cutoff_pair_count_matches_oracle(ctx):
    # the device count of pairs inside the cutoff (the algorithmic work of a pass) equals the oracle's
    # count exactly: both take the cutoff decision in the same FP32 operations
    xyz, v, L = W.fcc_modulated(16, 14, 14, 0.8442, 11000, seed=80)
    w = W.build_lj(xyz, W.two_types(xyz.shape[0], 8), L, 2.5, **W.LJ_TWO_TYPES)
    rig = LJRig(ctx, w)
    rig.b.reorganize(rig.pool, gc.REORG_NONE)
    got = rig.b.lj_count_pairs(w.rcut)
    _, _, want = O.lj_tasks(w, potential=True)
    assert got == want and got > 0
    rig.close()
