"""The C-ABI's error and resource contract on the device: allocator hooks, context poisoning, host-side
validation (overlapping direct ranges, node indices beyond the node table), and the device-side error
words (a whole-step wait that gives up, node ranges outside the id space in the adjoint's node chain).

Every failure here is forced from the host: the wait hook makes one step's waits give up after a few
probes (every wave still ends normally), and the bad node range is skipped by the kernel's own bounds
check.  Nothing is made to fault."""
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, grav_tasks, rel_l2_per_task, whole

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    return W.nbody_tiny()


def _run_tiny(c, w):
    import torch
    rig = GravRig(c, w)
    b = rig.batch(whole(w))
    ids, slots = W.residency(W.batch_union(whole(w)), w.n, 0.5, seed=3)
    rig.place(ids, slots)
    acc = rig.run(b, gc.REORG_PACK, order=1)
    torch.cuda.synchronize()
    b.destroy()
    rig.close()
    return acc


def test_allocator_hooks_take_every_device_buffer(tiny):
    # a context with the caller's allocator: the library's buffers come from it and all go back
    import torch
    live, calls = {}, {"alloc": 0, "free": 0}

    def alloc(nbytes, _user):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0)
        live[p] = nbytes
        calls["alloc"] += 1
        return p

    def free(p, _user):
        assert p in live
        del live[p]
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    print("[gpu] allocator hooks", flush=True)
    c = gc.Context(0, allocator=(alloc, free))
    acc = _run_tiny(c, tiny)
    assert calls["alloc"] >= 10, calls
    assert not live, f"{len(live)} buffers still held after the pool and batch were destroyed"
    c.close()
    ref = O.grav_workload(tiny, order=1)
    assert rel_l2_per_task(acc, ref, whole(tiny)).max() <= 1e-5


def test_torch_allocator_gives_the_same_bits(ctx, tiny):
    c = gc.Context(0, allocator="torch")
    got = _run_tiny(c, tiny)
    c.close()
    assert np.array_equal(got, _run_tiny(ctx, tiny))


def test_allocator_hooks_must_come_in_pairs():
    h = gc.VP()
    f = gc.ALLOC_FN(lambda n, u: None)
    st = gc.lib().gc_init(0, ctypes.cast(f, gc.VP), None, None, ctypes.byref(h))
    assert st == gc.GC_E_INVAL


def test_injected_error_poisons_the_context():
    # an asynchronous error (injected on the host; nothing reaches the device) surfaces as GC_E_HIP at
    # the next call; the context then answers GC_E_STATE until gc_finalize
    import torch
    c = gc.Context(0)
    buf = torch.zeros(16, device="cuda")
    c.zero(buf)
    c.inject_error(700)
    with pytest.raises(gc.GcError) as e:
        c.zero(buf)
    assert e.value.status == gc.GC_E_HIP
    assert "injected" in str(e.value)
    for _ in range(2):
        with pytest.raises(gc.GcError) as e:
            c.zero(buf)
        assert e.value.status == gc.GC_E_STATE
    out = gc.VP()
    assert gc.lib().gc_pool_create(c.h, 10, 10, ctypes.byref(out)) == gc.GC_E_STATE
    assert b"poisoned" in gc.lib().gc_last_error(c.h)
    c.close()


def test_overlapping_direct_ranges_are_rejected(ctx, tiny):
    b = gc.Batch(ctx, gc.KIND_GRAV, tiny.n)
    t = gc.tasks_from_csr([0], [4], [0], [2], [0], [0])
    for ranges in ([[10, 5], [12, 3]], [[10, 5], [10, 5]], [[20, 4], [10, 11]]):
        with pytest.raises(gc.GcError) as e:
            b.submit(t, np.array(ranges, np.int32))
        assert e.value.status == gc.GC_E_INVAL
        assert b.sizes()["tasks"] == 0  # nothing appended
    # touching and empty ranges are fine
    b.submit(t, np.array([[10, 5], [15, 3]], np.int32))
    b.submit(t, np.array([[10, 0], [10, 3]], np.int32))
    assert b.sizes()["tasks"] == 2
    b.destroy()


def test_node_index_beyond_the_table_is_rejected(ctx, tiny):
    import torch
    rig = GravRig(ctx, tiny)
    b = rig.batch(whole(tiny))
    b.reorganize(rig.pool, gc.REORG_NONE)
    top = int(tiny.node_idx.max())
    short = rig.nodes[:top].contiguous()  # node records 0 .. top-1: the largest index is out
    with pytest.raises(gc.GcError) as e:
        b.launch(gc.grav_params(order=1), short, rig.acc)
    assert e.value.status == gc.GC_E_INVAL
    s = torch.cuda.Stream()
    with pytest.raises(gc.GcError) as e:
        gc.Graph(ctx, [b], [rig.pool], [gc.REORG_NONE], gc.grav_params(order=1), short, rig.acc, stream=s)
    assert e.value.status == gc.GC_E_INVAL
    b.launch(gc.grav_params(order=1), rig.nodes, rig.acc)  # the whole table is fine
    torch.cuda.synchronize()
    b.destroy()
    rig.close()


def test_node_chain_skips_and_reports_out_of_range_nodes(ctx):
    # a node of the lists whose member range leaves [0, n_ids): the node chain skips it and the batch
    # reports GC_E_INVAL; the other nodes' gradients are unchanged
    import torch
    w = W.build_grav(W.plummer(4096, 61), bucket=16, theta=0.7)
    rig = GravRig(ctx, w)
    b = rig.batch(whole(w))
    rig.run(b, gc.REORG_NONE, order=2)
    b.status()
    g = np.random.default_rng(5).normal(size=(w.n, 3)).astype(np.float32)
    cot = torch.zeros((w.n, 4), dtype=torch.float32, device="cuda")
    cot[:, :3] = torch.from_numpy(g).cuda()
    nr_ok = np.ascontiguousarray(w.node_range).astype(np.int32)
    used = np.unique(w.node_idx)
    bad = int(used[len(used) // 2])
    nr_bad = nr_ok.copy()
    nr_bad[bad] = (w.n - 3, 10)
    outs = []
    for nr in (nr_ok, nr_bad):
        gpos = torch.zeros((w.n, 4), dtype=torch.float32, device="cuda")
        gmass = torch.zeros(w.n, dtype=torch.float32, device="cuda")
        b.backward(gc.grav_params(order=2), rig.nodes, torch.from_numpy(nr).cuda(), w.nodes.shape[0], cot, gpos,
                   gmass)
        torch.cuda.synchronize()
        outs.append(gpos.cpu().numpy())
    with pytest.raises(gc.GcError) as e:
        b.status()
    assert e.value.status == gc.GC_E_INVAL
    # the skipped node's members lose only its push: every particle outside it keeps its gradient (up to
    # the order of the FP32 atomic additions)
    lo, cnt = nr_ok[bad]
    inside = np.zeros(w.n, bool)
    inside[lo:lo + cnt] = True
    scale = np.abs(outs[0][:, :3]).max()
    assert np.abs(outs[0][~inside, :3] - outs[1][~inside, :3]).max() <= 1e-5 * scale
    b.destroy()
    rig.close()


def test_step_wait_that_gives_up_is_reported(ctx):
    # the test hook makes round 1's force items wait for one data part too many (a few probes each):
    # the launch ends normally and gc_graph_status reports it; with the hook off a new capture is clean
    import torch
    w = W.nbody_plummer(n=30000, seed=77)
    rig = GravRig(ctx, w)
    rounds = W.poisson_rounds(w.n_tasks, 500, seed=38)[:3]
    bs = [rig.batch(W.task_subset(w, r)) for r in rounds]
    ids, slots = W.residency(np.arange(w.n), w.n, 0.4, seed=39)
    rig.place(ids, slots)
    s = torch.cuda.Stream()
    sprm = gc.grav_params(order=2, schedule=gc.SCHED_STEP)
    print("[gpu] step wait hook: fail round 1 after 64 probes", flush=True)
    ctx.step_waits(fail_spins=64, fail_round=1)
    try:
        g = gc.Graph(ctx, bs, [rig.pool] * 3, [gc.REORG_PACK] * 3, sprm, rig.nodes, rig.acc, stream=s,
                     fixture=gc.FIXTURE_EVICT_STAGED)
    finally:
        ctx.step_waits(0, -1)
    g.launch(stream=s)
    with pytest.raises(gc.GcError) as e:
        g.status(stream=s)
    assert e.value.status == gc.GC_E_HIP
    with pytest.raises(gc.GcError):
        bs[1].status()
    g.destroy()
    # a capture without the hook clears the words; its launches report clean and match the oracle
    g = gc.Graph(ctx, bs, [rig.pool] * 3, [gc.REORG_PACK] * 3, sprm, rig.nodes, rig.acc, stream=s,
                 fixture=gc.FIXTURE_EVICT_STAGED)
    rig.acc.fill_(np.nan)
    torch.cuda.synchronize()
    g.launch(stream=s)
    g.status(stream=s)
    got = rig.acc.cpu().numpy()
    for r in rounds:
        bt = W.task_subset(w, r)
        assert rel_l2_per_task(got, O.grav_workload(w, order=2, tasks=bt), bt).max() <= 1e-5
    g.destroy()
    for b in bs:
        b.status()
        b.destroy()
    rig.close()


def test_deterministic_flag(ctx, tiny):
    # gravity forward sums without atomics: accepted, bitwise repeatable; its adjoint adds target
    # gradients with atomics: refused under the flag
    import torch
    rig = GravRig(ctx, tiny)
    b = rig.batch(whole(tiny))
    prm = gc.grav_params(order=1)
    prm.deterministic = 1
    a1 = rig.run(b, gc.REORG_PACK, order=1, deterministic=1)
    a2 = rig.run(b, gc.REORG_PACK, order=1, deterministic=1)
    assert np.array_equal(a1, a2)
    cot = torch.zeros((tiny.n, 4), device="cuda")
    gpos = torch.zeros((tiny.n, 4), device="cuda")
    gmass = torch.zeros(tiny.n, device="cuda")
    nr = torch.from_numpy(np.ascontiguousarray(tiny.node_range)).cuda()
    with pytest.raises(gc.GcError) as e:
        b.backward(prm, rig.nodes, nr, tiny.nodes.shape[0], cot, gpos, gmass)
    assert e.value.status == gc.GC_E_UNSUPPORTED
    b.destroy()
    rig.close()


def test_submit_copies_and_validates_against_grav_tasks(ctx, tiny):
    # the binding's task records reach the library unchanged (sizes agree with the submitted CSR)
    b = gc.Batch(ctx, gc.KIND_GRAV, tiny.n)
    t = whole(tiny)
    b.submit(grav_tasks(t), t["ranges"], t["node_idx"])
    sz = b.sizes()
    assert sz["tasks"] == tiny.n_tasks and sz["node_refs"] == tiny.node_idx.size
    assert sz["direct"] == int(np.asarray(t["ranges"])[:, 1].sum())
    b.destroy()
