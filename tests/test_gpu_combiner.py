"""The combining policy (Sec. 3.1) driving combined launches from a timestamped task stream.

Bucket tasks of nbody-uniform-4096 arrive in bursts on a simulated clock; at every poll the
requests the combiner takes leave the queue in arrival order, go into one batch and one combined
launch (PACK, the pool keeping half of all particles resident).  Every target is written by
exactly one launch, so the final accelerations must match the oracle's over the whole workload,
and no launch may hold more than max_size requests.
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, rel_l2_per_task, whole

pytestmark = pytest.mark.gpu


def test_combiner_drives_combined_launches():
    print("[gpu] combiner stream over nbody-uniform-4096", flush=True)
    ctx = gc.Context(0)
    w = W.nbody_tiny()
    rig = GravRig(ctx, w)
    bids, bslots = W.residency(np.arange(w.n, dtype=np.int32), w.n, 0.5, seed=21)
    rig.pool.reset()
    rig.place(bids, bslots)
    prm = gc.grav_params(order=1)
    per_cu, n_cu = ctx.occupancy(prm)
    assert per_cu >= 1 and n_cu >= 1  # the full-occupancy max_size a caller would use: per_cu * n_cu
    max_size = 64                     # smaller here, so that both rules fire on 539 tasks
    comb = gc.Combiner(max_size)
    rng = np.random.default_rng(22)
    T = w.n_tasks
    # bursts: 40 short gaps, then 10 long ones
    gaps = np.array([rng.exponential(1e-4 if k % 50 < 40 else 5e-3) for k in range(T)])
    times = np.cumsum(gaps)
    rig.acc.fill_(float("nan"))
    nxt, sizes, reasons = 0, [], []

    def launch(n):
        nonlocal nxt
        sel = np.arange(nxt, nxt + n)
        nxt += n
        b = rig.batch(W.task_subset(w, sel))
        b.reorganize(rig.pool, gc.REORG_PACK)
        b.launch(prm, rig.nodes, rig.acc)
        rig.pool.evict_staged(b)
        rig.torch.cuda.synchronize()
        b.destroy()

    t_poll = 0.0
    for i, t in enumerate(times):
        comb.arrive(float(t))
        t_next = times[i + 1] if i + 1 < T else t + 1.0
        while t_poll + 1e-3 < t_next:  # polls every millisecond of the simulated clock
            t_poll = max(t_poll + 1e-3, float(t))
            n, why = comb.poll(t_poll)
            if n:
                sizes.append(n)
                reasons.append(why)
                launch(n)
    n, why = comb.poll(float(times[-1]) + 10.0)
    if n:
        sizes.append(n)
        reasons.append(why)
        launch(n)
    assert nxt == T and comb.state()["waiting"] == 0
    assert max(sizes) <= max_size and 1 in reasons and 2 in reasons
    print(f"[gpu] {len(sizes)} launches, sizes {min(sizes)}..{max(sizes)}", flush=True)
    acc = rig.acc.cpu().numpy()
    err = rel_l2_per_task(acc, O.grav_workload(w, order=1), whole(w))
    assert err.max() <= 1e-5, err.max()
    comb.destroy()
    rig.close()
    ctx.close()
