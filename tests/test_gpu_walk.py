"""Device Barnes-Hut lists (gc_tree_walk) against the oracle walk: offsets, node lists and direct
ranges bit-exact, over the small workloads at several opening angles and the 262,144-particle
Plummer workload; an out-of-range bucket leaf is refused."""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def _dev(w, leaf=None):
    import torch
    leaf = w.meta["leaf"] if leaf is None else leaf
    return (torch.from_numpy(np.ascontiguousarray(w.node_range, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(w.node_mom64[:, :3])).cuda(),
            torch.from_numpy(np.ascontiguousarray(w.node_side)).cuda(),
            torch.from_numpy(np.ascontiguousarray(w.rec)).cuda(),
            torch.from_numpy(np.ascontiguousarray(leaf, np.int32)).cuda())


def _check(ctx, w, theta):
    import torch
    nf, nidx, rf, rng = gc.tree_walk(ctx, *_dev(w), theta)
    torch.cuda.synchronize()
    onf, onidx, orf, orng = O.bh_walk_workload(w, theta)
    assert np.array_equal(nf.cpu().numpy(), onf)
    assert np.array_equal(rf.cpu().numpy(), orf)
    assert np.array_equal(nidx.cpu().numpy(), onidx)
    assert np.array_equal(rng.cpu().numpy(), orng)
    return int(onf[-1]), int(orf[-1])


@pytest.mark.parametrize("theta", [0.0, 0.4, 0.7, 1.0])
def test_walk_matches_oracle_plummer_4096(ctx, theta):
    print(f"[gpu] tree walk, Plummer 4096 bucket 16, theta {theta}", flush=True)
    w = W.build_grav(W.plummer(4096, 61), bucket=16, theta=0.7)
    nn, nr = _check(ctx, w, theta)
    assert nr > 0 and (nn > 0) == (theta > 0)


def test_walk_matches_oracle_uniform_4096(ctx):
    print("[gpu] tree walk, uniform 4096", flush=True)
    _check(ctx, W.nbody_tiny(), 0.7)


def test_walk_matches_oracle_plummer_262144(ctx):
    print("[gpu] tree walk, Plummer 262144 bucket 32, theta 0.7", flush=True)
    w = W.nbody_plummer()
    nn, nr = _check(ctx, w, 0.7)
    assert nn == w.node_idx.shape[0] and nr == w.ranges.shape[0]


def test_walk_refuses_out_of_range_leaf(ctx):
    print("[gpu] tree walk, out-of-range bucket leaf", flush=True)
    w = W.nbody_tiny()
    leaf = w.meta["leaf"].astype(np.int32).copy()
    leaf[3] = w.nodes.shape[0]
    with pytest.raises(gc.GcError) as ei:
        gc.tree_walk(ctx, *_dev(w, leaf), 0.7)
    assert ei.value.status == gc.GC_E_INVAL
