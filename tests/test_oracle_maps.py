"""Pins for the checker's reorganisation maps.

The sorted index array is built by binary-search insertion in request order
(Sec. 3.2); here it is pinned to sort-unique, and every derived map is pinned
to a brute-force construction from Python sets on tiny random cases.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _random_batch(rng, n_ids, n_tasks, max_ranges=4, max_len=6):
    i_begin, i_count, j_first, j_nr, ranges = [], [], [], [], []
    for _ in range(n_tasks):
        c = min(int(rng.integers(1, 5)), n_ids)
        b = int(rng.integers(0, n_ids - c + 1))
        i_begin.append(b); i_count.append(c)
        j_first.append(len(ranges))
        k = int(rng.integers(0, max_ranges + 1))
        for _ in range(k):
            ln = int(rng.integers(1, max_len + 1))
            ln = min(ln, n_ids)
            s = int(rng.integers(0, n_ids - ln + 1))
            ranges.append((s, ln))
        j_nr.append(k)
    T = len(i_begin)
    return dict(i_begin=np.array(i_begin, np.int32), i_count=np.array(i_count, np.int32),
                n_first=np.zeros(T, np.int32), n_count=np.zeros(T, np.int32),
                j_first=np.array(j_first, np.int32), j_nr=np.array(j_nr, np.int32), node_idx=np.zeros(0, np.int32),
                ranges=np.array(ranges, np.int32).reshape(-1, 2))


def _brute(b, n_ids, cap, slot_of, mode):
    ids = set()
    for s, c in zip(b["i_begin"], b["i_count"]):
        ids.update(range(s, s + c))
    for s, c in b["ranges"]:
        ids.update(range(s, s + c))
    U = sorted(ids)
    pos = {u: k for k, u in enumerate(U)}
    so = list(slot_of)
    if mode == O.REDUNDANT:
        missing = list(U)
        new = []
    else:
        missing = [u for u in U if so[u] < 0]
        used = set(x for x in so if x >= 0)
        free = [s for s in range(cap) if s not in used]
        new = free[:len(missing)]
        for u, s in zip(missing, new):
            so[u] = s
    out = dict(U=U, missing=missing, new=new, slot_of=so)
    if mode in (O.REDUNDANT, O.PACK):
        out["pranges"] = [(pos[s], c) for s, c in b["ranges"]]
        out["pi_begin"] = [pos[s] for s in b["i_begin"]]
    else:
        il, jl = [], []
        for t in range(len(b["i_begin"])):
            il += [so[i] for i in range(b["i_begin"][t], b["i_begin"][t] + b["i_count"][t])]
            lst = []
            for s, c in b["ranges"][b["j_first"][t]:b["j_first"][t] + b["j_nr"][t]]:
                lst += [so[j] for j in range(s, s + c)]
            jl += sorted(lst) if mode == O.SORTED else lst
        out["ilist"], out["jlist"] = il, jl
    return out


@pytest.mark.parametrize("mode", [O.REDUNDANT, O.INDIRECT, O.SORTED, O.PACK])
def test_maps_brute_force_tiny(mode):
    rng = np.random.default_rng(100 + mode)
    for case in range(200):
        n_ids = int(rng.integers(1, 65))
        cap = int(rng.integers(n_ids, 2 * n_ids + 2))
        b = _random_batch(rng, n_ids, int(rng.integers(1, 9)))
        slot_of = np.full(n_ids, -1, np.int32)
        k = int(rng.integers(0, n_ids + 1))
        res = rng.choice(n_ids, size=k, replace=False)
        slot_of[res] = rng.choice(cap, size=k, replace=False)
        got = O.maps(b, n_ids, cap, slot_of, mode)
        want = _brute(b, n_ids, cap, slot_of, mode)
        assert got["status"] == 0
        assert got["U"].tolist() == want["U"], case
        assert got["missing"].tolist() == want["missing"]
        if mode != O.REDUNDANT:
            assert got["new_slot"].tolist() == want["new"]
            assert got["slot_of"].tolist() == want["slot_of"]
        else:
            assert got["slot_of"].tolist() == slot_of.tolist()
        if mode in (O.REDUNDANT, O.PACK):
            assert [tuple(x) for x in got["pranges"].tolist()] == want["pranges"]
            assert got["pi_begin"].tolist() == want["pi_begin"]
        else:
            assert got["ilist"].tolist() == want["ilist"]
            assert got["jlist"].tolist() == want["jlist"]


def test_pool_full_reported():
    b = dict(i_begin=np.array([0], np.int32), i_count=np.array([4], np.int32), n_first=np.zeros(1, np.int32),
             n_count=np.zeros(1, np.int32), j_first=np.zeros(1, np.int32), j_nr=np.zeros(1, np.int32),
             node_idx=np.zeros(0, np.int32), ranges=np.zeros((0, 2), np.int32))
    slot_of = np.array([-1, -1, -1, -1, 0, 1], np.int32)
    assert O.maps(b, 6, 5, slot_of, O.PACK)["status"] == 3
    assert O.maps(b, 6, 6, slot_of, O.PACK)["status"] == 0


def test_insertion_union_equals_sort_unique_on_tree_rounds():
    w = W.nbody_plummer(n=20000, seed=41)
    for r in W.poisson_rounds(w.n_tasks, 300, seed=42)[:3]:
        b = W.task_subset(w, r)
        U = O.union_insert(b, w.n)
        assert np.array_equal(U, W.batch_union(b))


def test_packed_ranges_are_contiguous_images():
    # a range [b, b+c) of ids maps to [pos[b], pos[b]+c): every id inside is in U, so ranks are consecutive
    w = W.nbody_plummer(n=20000, seed=43)
    b = W.task_subset(w, np.arange(0, 200))
    m = O.maps(b, w.n, w.n, np.full(w.n, -1, np.int32), O.PACK)
    pos = m["pos"]
    for (s, c), (ps, pc) in zip(b["ranges"], m["pranges"]):
        assert pc == c and np.array_equal(pos[s:s + c], np.arange(ps, ps + c))
