"""Device-side submission and commit: the list walk's output becomes combined requests without leaving
the device (gc_tree_walk -> gc_walk_tasks -> gc_submit_tasks_device -> gc_batch_commit).

Bars: the union U, every position in it and the packed-space maps bit-exact against the oracle's
binary-search insertion (Sec. 3.2); reorganisation maps bit-exact; forces bitwise equal to those of
the same request submitted from the host, and within per-task relative L2 1e-5 of the oracle; a
submission outside the device contract is refused at commit.
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, rel_l2_per_task, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def plum():
    return W.nbody_plummer(n=30000, seed=77)


def walk(ctx, w):
    torch = torch_cuda()
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
           (w.node_range.astype(np.int32), w.node_mom64[:, :3], w.node_side, w.rec, w.meta["leaf"].astype(np.int32))]
    nf, nidx, rf, rng = gc.tree_walk(ctx, *dev, w.theta)
    return dev, nf, nidx, rf, rng


def device_batch(ctx, w, walked, b0, b1):
    dev, nf, nidx, rf, rng = walked
    nfh, rfh = nf.cpu().numpy(), rf.cpu().numpy()
    tasks = gc.walk_tasks(ctx, b0, b1, dev[4], dev[0], nf, rf)
    b = gc.Batch(ctx, gc.KIND_GRAV, w.n)
    b.submit_device(tasks, rng[rfh[b0]:rfh[b1]], nidx[nfh[b0]:nfh[b1]], w.nodes.shape[0])
    b.commit()
    return b


@pytest.mark.parametrize("mode", [gc.REORG_PACK, gc.REORG_INDIRECT, gc.REORG_SORTED])
def test_device_commit_maps_bit_exact(ctx, plum, mode):
    print(f"[gpu] device commit maps mode={mode}", flush=True)
    walked = walk(ctx, plum)
    rig = GravRig(ctx, plum)
    for k, (b0, b1) in enumerate([(0, 1), (1000, 1700), (plum.n_tasks - 333, plum.n_tasks)]):
        bt = W.task_subset(plum, np.arange(b0, b1))
        ids, slots = W.residency(W.batch_union(bt), plum.n, 0.5, seed=20 + k)
        rig.pool.reset()
        rig.place(ids, slots)
        before = rig.pool.query()
        b = device_batch(ctx, plum, walked, b0, b1)
        assert b.sizes() == dict(tasks=b1 - b0, ranges=int(bt["ranges"].shape[0]), node_refs=int(bt["node_idx"].size),
                                 direct=int(bt["ranges"][:, 1].sum()), targets=int(bt["i_count"].sum()))
        b.reorganize(rig.pool, mode)
        got = b.maps()
        want = O.maps(bt, plum.n, plum.n, before, mode)
        assert want["status"] == 0
        assert np.array_equal(got["U"], O.union_insert(bt, plum.n))
        assert np.array_equal(got["U"], want["U"])
        assert np.array_equal(got["pos"], want["pos"])
        assert np.array_equal(got["missing"], want["missing"])
        assert np.array_equal(got["new_slot"], want["new_slot"])
        assert np.array_equal(rig.pool.query(), want["slot_of"])
        if mode == gc.REORG_PACK:
            assert np.array_equal(got["pranges"], want["pranges"])
            assert np.array_equal(got["pi_begin"], want["pi_begin"])
        else:
            assert np.array_equal(got["ilist"], want["ilist"])
            assert np.array_equal(got["jlist"], want["jlist"])
        b.destroy()
    rig.close()


def test_device_commit_forces_equal_host_commit(ctx, plum):
    # every Poisson round of the workload, committed on the device from the walk and on the host from
    # the generator's lists: the same bits, and the oracle's forces
    torch = torch_cuda()
    print("[gpu] device commit forces, all rounds", flush=True)
    walked = walk(ctx, plum)
    rig = GravRig(ctx, plum)
    rounds = W.poisson_rounds(plum.n_tasks, 400, seed=31)
    ref = O.grav_workload(plum, order=2)
    prm = gc.grav_params(order=2)
    accd = torch.full((plum.n, 4), float("nan"), device="cuda")
    acch = torch.full((plum.n, 4), float("nan"), device="cuda")
    for r in rounds:
        b0, b1 = int(r[0]), int(r[-1]) + 1
        bd = device_batch(ctx, plum, walked, b0, b1)
        bh = rig.batch(W.task_subset(plum, r))
        for b, acc in ((bd, accd), (bh, acch)):
            b.reorganize(rig.pool, gc.REORG_PACK, check_capacity=False)
            b.launch(prm, rig.nodes, acc)
            rig.pool.evict_staged(b)
        bd.destroy()
        bh.destroy()
    torch.cuda.synchronize()
    a_d, a_h = accd.cpu().numpy(), acch.cpu().numpy()
    assert np.array_equal(a_d, a_h)
    err = rel_l2_per_task(a_d, ref, W.task_subset(plum, np.arange(plum.n_tasks)))
    assert err.max() <= TOL, err.max()
    rig.close()


def test_device_commit_graph_capture_uses_device_order(ctx, plum):
    # a whole-step capture of device-committed rounds (the host copies their lists once) gives the
    # per-round launches' bits
    torch = torch_cuda()
    walked = walk(ctx, plum)
    rig = GravRig(ctx, plum)
    rounds = W.poisson_rounds(plum.n_tasks, 400, seed=32)[:5]
    bs = [device_batch(ctx, plum, walked, int(r[0]), int(r[-1]) + 1) for r in rounds]
    prm = gc.grav_params(order=2, schedule=gc.SCHED_STEP)
    g = gc.Graph(ctx, bs, [rig.pool] * len(bs), [gc.REORG_PACK] * len(bs), prm, rig.nodes, rig.acc,
                 stream=torch.cuda.Stream(), fixture=gc.FIXTURE_EVICT_STAGED)
    rig.acc.fill_(float("nan"))
    g.launch()
    torch.cuda.synchronize()
    g.status()
    step = rig.acc.cpu().numpy()
    g.destroy()
    ref = torch.full_like(rig.acc, float("nan"))
    for b in bs:
        b.reorganize(rig.pool, gc.REORG_PACK, check_capacity=False)
        b.launch(gc.grav_params(order=2), rig.nodes, ref)
        rig.pool.evict_staged(b)
    torch.cuda.synchronize()
    tgt = np.concatenate([np.arange(plum.i_begin[t], plum.i_begin[t] + plum.i_count[t])
                          for r in rounds for t in r])
    assert np.array_equal(step[tgt], ref.cpu().numpy()[tgt])
    for b in bs:
        b.destroy()
    rig.close()


def test_empty_device_submission(ctx, plum):
    torch = torch_cuda()
    rig = GravRig(ctx, plum)
    b = gc.Batch(ctx, gc.KIND_GRAV, plum.n)
    z = torch.zeros(0, dtype=torch.int32, device="cuda")
    b.submit_device(torch.zeros(0, dtype=torch.uint8, device="cuda"), z, z, plum.nodes.shape[0])
    b.commit()
    assert b.sizes()["tasks"] == 0
    b.reorganize(rig.pool, gc.REORG_PACK)
    b.launch(gc.grav_params(order=2), rig.nodes, rig.acc)
    torch.cuda.synchronize()
    assert b.maps()["U"].size == 0
    b.destroy()
    rig.close()


@pytest.mark.parametrize("fault", ["descending", "node", "targets", "slice", "mixed"])
def test_device_submission_contract(ctx, plum, fault):
    torch = torch_cuda()
    bt = W.task_subset(plum, np.arange(200, 260))
    tasks = gc.tasks_from_csr(bt["i_begin"], bt["i_count"], bt["j_first"], bt["j_nr"], bt["n_first"], bt["n_count"])
    ranges = bt["ranges"].copy()
    nodes = bt["node_idx"].copy()
    if fault == "descending":
        t = int(np.argmax(bt["j_nr"] >= 2))
        f = bt["j_first"][t]
        ranges[[f, f + 1]] = ranges[[f + 1, f]]
    elif fault == "node":
        nodes[5] = plum.nodes.shape[0]
    elif fault == "targets":
        tasks["i_begin"][7] = tasks["i_begin"][6]
        tasks["i_count"][7] = tasks["i_count"][6]
    elif fault == "slice":
        tasks["j_nranges"][3] = ranges.shape[0]
    b = gc.Batch(ctx, gc.KIND_GRAV, plum.n)
    dt = torch.from_numpy(tasks.view(np.uint8).copy()).cuda()
    b.submit_device(dt, torch.from_numpy(ranges).cuda(), torch.from_numpy(nodes).cuda(), plum.nodes.shape[0])
    if fault == "mixed":
        with pytest.raises(gc.GcError) as e:
            b.submit(tasks, ranges, nodes)
        assert e.value.status == gc.GC_E_STATE
        b.commit()
    else:
        with pytest.raises(gc.GcError) as e:
            b.commit()
        assert e.value.status == gc.GC_E_INVAL
    b.destroy()
