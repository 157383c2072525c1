"""Pins of the oracle's Barnes-Hut list walk (oracle.bh_walk).

Checked against: the input generator's lists (a separate, stack-based walk of the same definition),
the partition property (a bucket's accepted nodes and direct ranges cover every id once), the
opening test recomputed for every accepted node and every direct leaf, and theta = 0 (nothing is
accepted: every leaf is direct).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _plummer():
    return W.build_grav(W.plummer(4096, 61), bucket=16, theta=0.7)


def _dist(com, lo, hi):
    e = np.where(com < lo, lo - com, np.where(com > hi, com - hi, 0.0))
    return np.sqrt((e[..., 0] * e[..., 0] + e[..., 1] * e[..., 1]) + e[..., 2] * e[..., 2])


@pytest.mark.parametrize("make", [W.nbody_tiny, _plummer])
def test_walk_matches_generator_lists(make):
    w = make()
    nf, nidx, rf, rng = O.bh_walk_workload(w)
    assert np.array_equal(nf[:-1], w.n_first) and np.array_equal(np.diff(nf), w.n_count)
    assert np.array_equal(nidx, w.node_idx)
    assert np.array_equal(rf[:-1], w.j_first) and np.array_equal(np.diff(rf), w.j_nr)
    assert np.array_equal(rng, w.ranges)


@pytest.mark.parametrize("theta", [0.4, 0.7, 1.0])
def test_walk_partitions_ids_and_obeys_the_opening_test(theta):
    w = _plummer()
    nf, nidx, rf, rng = O.bh_walk_workload(w, theta)
    leaf = w.meta["leaf"]
    com = w.node_mom64[:, :3]
    children = np.bincount(w.node_parent[1:], minlength=w.nodes.shape[0])
    for b in range(0, leaf.shape[0], 7):
        bf, bc = w.node_range[leaf[b]]
        pos = w.rec[bf:bf + bc, :3].astype(np.float64)
        lo, hi = pos.min(0), pos.max(0)
        nodes = nidx[nf[b]:nf[b + 1]]
        direct = rng[rf[b]:rf[b + 1]]
        spans = np.concatenate([w.node_range[nodes], direct]) if len(nodes) else direct
        order = np.argsort(spans[:, 0], kind="stable")
        s = spans[order]
        assert s[0, 0] == 0 and s[-1].sum() == w.n and np.array_equal(s[1:, 0], s[:-1].sum(1))
        # accepted: disjoint from the bucket and side < theta * dist
        nr = w.node_range[nodes]
        assert np.all((nr[:, 0] + nr[:, 1] <= bf) | (bf + bc <= nr[:, 0]))
        assert np.all(w.node_side[nodes] < theta * _dist(com[nodes], lo, hi))
        # direct: leaves that overlap the bucket or fail the test
        dl = np.searchsorted(w.node_range[leaf, 0], direct[:, 0])
        dn = leaf[dl]
        assert np.array_equal(w.node_range[dn], direct) and np.all(children[dn] == 0)
        overlap = ~((direct[:, 0] + direct[:, 1] <= bf) | (bf + bc <= direct[:, 0]))
        assert np.all(overlap | ~(w.node_side[dn] < theta * _dist(com[dn], lo, hi)))


def test_walk_theta_zero_takes_no_node():
    w = W.nbody_tiny()
    nf, nidx, rf, rng = O.bh_walk_workload(w, 0.0)
    leaf = w.meta["leaf"]
    assert nf[-1] == 0 and nidx.size == 0
    assert np.all(np.diff(rf) == leaf.shape[0])
    for b in range(leaf.shape[0]):
        assert np.array_equal(rng[rf[b]:rf[b + 1]], w.node_range[leaf])
