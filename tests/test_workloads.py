"""Invariants of the seeded inputs: tree order, list coverage, acceptance rule, cell tasks."""
import numpy as np

import workloads as W


def _cover_counts(w, t):
    cov = np.zeros(w.n, np.int32)
    for k in w.node_idx[w.n_first[t]:w.n_first[t] + w.n_count[t]]:
        b, c = w.node_range[k]
        cov[b:b + c] += 1
    for b, c in w.ranges[w.j_first[t]:w.j_first[t] + w.j_nr[t]]:
        cov[b:b + c] += 1
    return cov


def test_tree_relabel_and_buckets():
    w = W.nbody_plummer(n=30000, seed=21)
    assert np.array_equal(np.sort(w.perm), np.arange(w.n))
    assert np.all(w.i_count <= w.bucket) and np.all(w.i_count >= 1)
    # buckets tile [0, N) in order
    assert w.i_begin[0] == 0 and np.all(w.i_begin[1:] == w.i_begin[:-1] + w.i_count[:-1])
    assert w.i_begin[-1] + w.i_count[-1] == w.n
    # children ranges nest inside parents
    par = w.node_parent
    nr = w.node_range
    ok = par < 0
    p = par[~ok]
    c = np.nonzero(~ok)[0]
    assert np.all(nr[c, 0] >= nr[p, 0]) and np.all(nr[c, 0] + nr[c, 1] <= nr[p, 0] + nr[p, 1])


def test_list_coverage_partition():
    # every bucket's nodes and direct ranges cover [0, N) exactly once
    w = W.nbody_plummer(n=20000, seed=22)
    rng = np.random.default_rng(0)
    for t in rng.choice(w.n_tasks, size=60, replace=False):
        assert np.all(_cover_counts(w, t) == 1)
    w0 = W.build_grav(W.uniform_cube(2000, 23), 16, theta=0.0)
    for t in range(0, w0.n_tasks, 7):
        assert np.all(_cover_counts(w0, t) == 1)


def test_acceptance_rule_and_minimality():
    w = W.nbody_plummer(n=20000, seed=24)
    rec = w.rec.astype(np.float64)
    com = w.node_mom64[:, :3]
    rng = np.random.default_rng(1)
    for t in rng.choice(w.n_tasks, size=40, replace=False):
        b, c = w.i_begin[t], w.i_count[t]
        lo, hi = rec[b:b + c, :3].min(0), rec[b:b + c, :3].max(0)

        def dist(k):
            e = np.maximum(0, np.maximum(lo - com[k], com[k] - hi))
            return np.linalg.norm(e)

        def acceptable(k):
            nb, nc = w.node_range[k]
            disjoint = nb + nc <= b or b + c <= nb
            return disjoint and w.node_side[k] < w.theta * dist(k)

        for k in w.node_idx[w.n_first[t]:w.n_first[t] + w.n_count[t]]:
            assert acceptable(k)
            p = w.node_parent[k]
            assert p < 0 or not acceptable(p)


def test_cell_tasks_cover_each_pair_once():
    w = W.lj_small()
    nc = int(np.prod(w.ncell))
    assert w.n_tasks == 14 * nc
    cell_of = np.empty(w.n, np.int64)
    for c in range(nc):
        cell_of[w.cell_start[c]:w.cell_start[c + 1]] = c
    seen = {}
    for t in range(w.n_tasks):
        a = cell_of[w.i_begin[t]] if w.i_count[t] else None
        bcell = cell_of[w.j_begin[t]] if w.j_count[t] else None
        key = (t // 14, int(np.searchsorted(w.cell_start, w.j_begin[t], side="right") - 1))
        if w.self_flag[t]:
            assert key[0] == key[1]
        pair = tuple(sorted(key))
        seen[pair] = seen.get(pair, 0) + 1
        del a, bcell
    assert all(v == 1 for v in seen.values())
    assert len(seen) == 14 * nc


def test_lj_lattice_counts():
    xyz, v, L = W.fcc_modulated(6, 5, 5, 0.8442, 500, seed=3)
    assert xyz.shape == (500, 3)
    np.testing.assert_allclose(np.sum(v * v) / (3 * 499), 1.0, rtol=1e-12)
    np.testing.assert_allclose(v.mean(0), 0, atol=1e-12)


def test_rounds_and_residency():
    r = W.poisson_rounds(1000, 50.0, seed=5)
    assert np.array_equal(np.concatenate(r), np.arange(1000))
    U = np.arange(10, 110)
    ids, slots = W.residency(U, 500, 0.5, seed=6)
    assert ids.size == 50 and np.unique(ids).size == 50 and np.all(np.isin(ids, U))
    assert np.unique(slots).size == 50 and slots.max() < 500


def test_wrapped_rounds_are_consecutive_modulo_the_task_count():
    one = W.poisson_rounds(27026, 2048, seed=1002)
    many = W.poisson_rounds(27026, 2048, seed=1002, n_rounds=32)
    assert len(many) == 32
    flat = np.concatenate(many)
    # consecutive tasks in tree order, wrapping from the last task to the first
    assert np.all(np.diff(flat) % 27026 == 1)
    assert flat[0] == 0
    # the rounds before the first wrap are those of the single pass
    k = 0
    while many[k][-1] >= many[k][0] and k + 1 < len(one):
        assert np.array_equal(many[k], one[k])
        k += 1
    assert k >= 12
