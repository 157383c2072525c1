"""Host-issued staging copies of the missing records (gc_pool_set_host_source, gc_reorganize's side stream).

The host finds each request's missing records in its mirror of the chare table, packs them into a
pinned buffer and copies them in on a side stream; the reorganisation kernel takes them from there
(Sec. 2.2, Sec. 3.2: only data not already on the device is transferred).  Bars: maps bit-exact
against the oracle; the host mirror equal to the device's chare table after every call; forces
bitwise equal to those of a device-source pool and within per-task relative L2 1e-5 of the oracle.
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, grav_tasks, rel_l2_per_task, torch_cuda, whole

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


def host_rig(ctx, w, capacity=None):
    rig = GravRig(ctx, w, capacity)
    rig.host = np.ascontiguousarray(w.rec, dtype=np.float32)
    rig.pool.set_host_source(rig.host)
    return rig


@pytest.mark.parametrize("side", [False, True])
@pytest.mark.parametrize("mode", [gc.REORG_PACK, gc.REORG_INDIRECT, gc.REORG_SORTED, gc.REORG_REDUNDANT])
def test_host_staged_maps_bit_exact(ctx, plum, mode, side):
    torch = torch_cuda()
    print(f"[gpu] host-staged maps mode={mode} side={side}", flush=True)
    rig = host_rig(ctx, plum)
    bt = W.task_subset(plum, np.arange(1000, 1700))
    ids, slots = W.residency(W.batch_union(bt), plum.n, 0.5, seed=9)
    rig.pool.reset()
    rig.place(ids, slots)
    before = rig.pool.query()
    assert np.array_equal(rig.pool.query_mirror(), before)
    b = rig.batch(bt)
    ss = torch.cuda.Stream() if side else None
    b.reorganize(rig.pool, mode, side=ss)
    got = b.maps()
    after = rig.pool.query()
    want = O.maps(bt, plum.n, plum.n, before, mode)
    assert want["status"] == 0
    assert np.array_equal(got["U"], want["U"])
    assert np.array_equal(got["pos"], want["pos"])
    assert np.array_equal(got["missing"], want["missing"])
    assert np.array_equal(after, want["slot_of"])
    assert np.array_equal(rig.pool.query_mirror(), after)
    if mode != gc.REORG_REDUNDANT:
        assert np.array_equal(got["new_slot"], want["new_slot"])
    if mode in (gc.REORG_PACK, gc.REORG_REDUNDANT):
        assert np.array_equal(got["pranges"], want["pranges"])
        assert np.array_equal(got["pi_begin"], want["pi_begin"])
    else:
        assert np.array_equal(got["ilist"], want["ilist"])
        assert np.array_equal(got["jlist"], want["jlist"])
    b.destroy()
    rig.close()


@pytest.mark.parametrize("mode", [gc.REORG_PACK, gc.REORG_INDIRECT, gc.REORG_REDUNDANT])
def test_rounds_with_eviction_match_device_source_bitwise(ctx, plum, mode):
    # the bench's fixture: a base residency of half of all ids; each round evicts what the round before
    # staged; round r's copy overlaps round r-1's pass (side stream).  Same rounds on a device-source
    # pool: the same maps and so the same bits
    torch = torch_cuda()
    print(f"[gpu] host-staged rounds mode={mode}", flush=True)
    rounds = W.poisson_rounds(plum.n_tasks, 300, seed=11)[:6]
    bids, bslots = W.residency(np.arange(plum.n, dtype=np.int32), plum.n, 0.5, seed=12)
    ref = O.grav_workload(plum, order=2)
    prm = gc.grav_params(order=2)
    out = {}
    for host in (True, False):
        rig = host_rig(ctx, plum) if host else GravRig(ctx, plum)
        rig.pool.reset()
        rig.place(bids, bslots)
        side = torch.cuda.Stream()
        bs = [rig.batch(W.task_subset(plum, r)) for r in rounds]
        accs = [torch.full((plum.n, 4), float("nan"), device="cuda") for _ in rounds]
        for k, b in enumerate(bs):
            if k:
                rig.pool.evict_staged(bs[k - 1])
            b.reorganize(rig.pool, mode, check_capacity=False, side=side if host else None)
            b.launch(prm, rig.nodes, accs[k])
            if host and k % 2:
                # the device's table after this round's eviction and staging equals the host's mirror
                assert np.array_equal(rig.pool.query_mirror(), rig.pool.query()), k
        torch.cuda.synchronize()
        out[host] = [a.cpu().numpy() for a in accs]
        if host:
            rig.pool.evict_staged(bs[-1])
            assert np.array_equal(rig.pool.query_mirror(), rig.pool.query())
        for b in bs:
            b.status()
            b.destroy()
        rig.close()
    for k, r in enumerate(rounds):
        bt = W.task_subset(plum, r)
        tgt = np.concatenate([np.arange(s, s + c) for s, c in zip(bt["i_begin"], bt["i_count"])])
        assert np.array_equal(out[True][k][tgt], out[False][k][tgt]), k
        err = rel_l2_per_task(out[True][k], ref, bt)
        assert err.max() <= TOL, (k, err.max())


def test_repeated_calls_reuse_the_pinned_buffer(ctx, plum):
    # the same batch reorganised and launched again and again (its pinned buffer and staged records
    # reused): every pass the same bits
    torch = torch_cuda()
    rig = host_rig(ctx, plum)
    bt = W.task_subset(plum, np.arange(0, 900))
    ids, slots = W.residency(W.batch_union(bt), plum.n, 0.5, seed=3)
    rig.pool.reset()
    rig.place(ids, slots)
    b = rig.batch(bt)
    side = torch.cuda.Stream()
    prm = gc.grav_params(order=1)
    first = None
    for rep in range(5):
        rig.acc.fill_(float("nan"))
        b.reorganize(rig.pool, gc.REORG_PACK, side=side)
        b.launch(prm, rig.nodes, rig.acc)
        rig.pool.evict_staged(b)
        got = rig.acc.cpu().numpy()
        if first is None:
            first = got
            err = rel_l2_per_task(got, O.grav_workload(plum, order=1, tasks=bt), bt)
            assert err.max() <= TOL
        else:
            assert np.array_equal(got, first, equal_nan=True), rep
    assert np.array_equal(rig.pool.query_mirror(), rig.pool.query())
    b.destroy()
    rig.close()


def test_mirror_is_read_back_after_device_source_work(ctx, plum):
    # device-source reorganisations change the table without the host; after switching to a host
    # source the first call reads the table back, and its maps still match the oracle
    rig = GravRig(ctx, plum)
    rig.pool.reset()
    bt0 = W.task_subset(plum, np.arange(0, 500))
    b0 = rig.batch(bt0)
    b0.reorganize(rig.pool, gc.REORG_PACK)
    host = np.ascontiguousarray(plum.rec, dtype=np.float32)
    rig.pool.set_host_source(host)
    before = rig.pool.query()
    bt = W.task_subset(plum, np.arange(300, 1100))
    b = rig.batch(bt)
    b.reorganize(rig.pool, gc.REORG_PACK)
    got = b.maps()
    want = O.maps(bt, plum.n, plum.n, before, gc.REORG_PACK)
    assert np.array_equal(got["missing"], want["missing"])
    assert np.array_equal(got["new_slot"], want["new_slot"])
    assert np.array_equal(rig.pool.query(), want["slot_of"])
    assert np.array_equal(rig.pool.query_mirror(), want["slot_of"])
    for x in (b0, b):
        x.destroy()
    rig.close()


def test_capacity_check_uses_the_mirror(ctx, plum):
    rig = host_rig(ctx, plum, capacity=1000)
    rig.pool.reset()
    bt = W.task_subset(plum, np.arange(0, 200))
    b = rig.batch(bt)
    before = rig.pool.query()
    with pytest.raises(gc.GcError) as e:
        b.reorganize(rig.pool, gc.REORG_PACK)
    assert e.value.status == 3
    assert np.array_equal(rig.pool.query(), before)
    assert np.array_equal(rig.pool.query_mirror(), before)
    b.destroy()
    rig.close()


def test_host_source_refusals(ctx, plum):
    torch = torch_cuda()
    rig = host_rig(ctx, plum)
    bt = W.task_subset(plum, np.arange(0, 100))
    b = rig.batch(bt)
    with pytest.raises(gc.GcError) as e:
        b.reorganize(rig.pool, gc.REORG_NONE)
    assert e.value.status == 1
    with pytest.raises(gc.GcError) as e:
        gc.Graph(ctx, [b], [rig.pool], [gc.REORG_PACK], gc.grav_params(order=2), rig.nodes, rig.acc,
                 stream=torch.cuda.Stream())
    assert e.value.status == 6
    with pytest.raises(gc.GcError) as e:
        rig.place(np.array([plum.n + 5]), np.array([0]))
    assert e.value.status == 1
    b.destroy()
    rig.close()
