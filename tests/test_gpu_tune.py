"""The autotuner's aggregation count and tuning cache (gc_autotune), and aggregated launches.

Bars: a batch split into consecutive launches of k tasks gives the same bits as one launch (each task's
sums do not depend on the launch it runs in); the tuned parameters reproduce the oracle's forces within
per-task relative L2 1e-5; the cache returns the stored entry without timing and keeps other entries;
a file that is not a cache is refused and left unchanged.
"""
import json

import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W
from gpu_helpers import GravRig, rel_l2_per_task, torch_cuda, whole

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


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("mode", [gc.REORG_PACK, gc.REORG_INDIRECT])
def test_aggregated_launches_are_bitwise_equal(ctx, plum, schedule, mode):
    torch = torch_cuda()
    rig = GravRig(ctx, plum)
    b = rig.batch(whole(plum))
    b.reorganize(rig.pool, mode)
    outs = []
    for agg in (0, 1, 7, 1000, plum.n_tasks - 1, plum.n_tasks + 5):
        rig.acc.fill_(float("nan"))
        b.launch(gc.grav_params(order=2, schedule=schedule, aggregation=agg), rig.nodes, rig.acc)
        torch.cuda.synchronize()
        outs.append(rig.acc.cpu().numpy())
    for k, o in enumerate(outs[1:]):
        assert np.array_equal(o, outs[0]), k
    err = rel_l2_per_task(outs[0], O.grav_workload(plum, order=2), whole(plum))
    assert err.max() <= TOL
    b.destroy()
    rig.close()


def test_autotune_cache(ctx, plum, tmp_path):
    torch = torch_cuda()
    rig = GravRig(ctx, plum)
    bt = W.task_subset(plum, np.arange(0, 2000))
    b = rig.batch(bt)
    b.reorganize(rig.pool, gc.REORG_PACK)
    path = str(tmp_path / "tune.json")
    best, times, hit = b.autotune(gc.grav_params(order=2), rig.nodes, rig.acc, reps=2, cache_path=path)
    assert not hit and np.all(np.isfinite(times)) and np.all(times > 0)
    entries = json.load(open(path))
    assert len(entries) == 1
    (key, ent), = entries.items()
    assert key.startswith("gfx") and ":grav_quad:" in key
    assert (ent["tile"], ent["waves_per_block"], ent["schedule"], ent["targets_per_lane"], ent["aggregation"]) == \
        (best.tile, best.waves_per_block, best.schedule, best.targets_per_lane, best.aggregation)
    best2, times2, hit2 = b.autotune(gc.grav_params(order=2), rig.nodes, rig.acc, reps=2, cache_path=path)
    assert hit2 and np.all(np.isnan(times2))
    assert (best2.tile, best2.waves_per_block, best2.schedule, best2.targets_per_lane, best2.aggregation) == \
        (best.tile, best.waves_per_block, best.schedule, best.targets_per_lane, best.aggregation)
    # the tuned parameters reproduce the oracle's forces
    rig.acc.fill_(float("nan"))
    b.launch(best2, rig.nodes, rig.acc)
    torch.cuda.synchronize()
    err = rel_l2_per_task(rig.acc.cpu().numpy(), O.grav_workload(plum, order=2, tasks=bt), bt)
    assert err.max() <= TOL
    # another batch shape and the monopole kernel get keys of their own; the first entry is kept
    b2 = rig.batch(W.task_subset(plum, np.arange(2000, 3000)))
    b2.reorganize(rig.pool, gc.REORG_PACK)
    _, _, hit3 = b2.autotune(gc.grav_params(order=1), rig.nodes, rig.acc, reps=1, cache_path=path)
    assert not hit3
    entries2 = json.load(open(path))
    assert len(entries2) == 2 and entries2[key] == ent
    b2.destroy()
    b.destroy()
    rig.close()


def test_autotune_refuses_a_foreign_file(ctx, plum, tmp_path):
    rig = GravRig(ctx, plum)
    b = rig.batch(W.task_subset(plum, np.arange(0, 100)))
    b.reorganize(rig.pool, gc.REORG_PACK)
    path = tmp_path / "notes.json"
    path.write_text('{"something": [1, 2, 3]}\n')
    with pytest.raises(gc.GcError) as e:
        b.autotune(gc.grav_params(order=2), rig.nodes, rig.acc, reps=1, cache_path=str(path))
    assert e.value.status == gc.GC_E_INVAL
    assert path.read_text() == '{"something": [1, 2, 3]}\n'
    b.destroy()
    rig.close()
