"""Reorganisation of large pools: the wide free-slot scan (a launch of its own, 64 slots a thread)
ahead of the union blocks (Sec. 3.2: the k-th missing record takes the k-th lowest free slot).

Bars: U, every position, the missing list, the new slots, the packed-space maps and the chare table
afterwards bit-exact against the oracle's maps on the same pool state; a second call after evicting
the first call's staging gives the same maps again (the wide scan's counters and tags rewind).
"""
import numpy as np
import pytest

import oracle as O
import paper_2008_05712_amd as gc
from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu

N = 1 << 22      # ids and pool slots: 1,024 narrow free-scan blocks, so the wide scan runs
RUN = 64


@pytest.fixture(scope="module")
def ctx():
    c = gc.Context(0)
    yield c
    c.close()


def _runs(rng, n_runs):
    starts = np.sort(rng.choice(N // RUN, size=n_runs, replace=False)).astype(np.int64) * RUN
    tasks = dict(i_begin=starts.astype(np.int32), i_count=np.full(n_runs, RUN, np.int32),
                 j_first=np.zeros(n_runs, np.int32), j_nr=np.zeros(n_runs, np.int32),
                 n_first=np.zeros(n_runs, np.int32), n_count=np.zeros(n_runs, np.int32),
                 ranges=np.zeros((0, 2), np.int32), node_idx=np.zeros(0, np.int32))
    union = (starts[:, None] + np.arange(RUN)[None, :]).reshape(-1)
    return tasks, union


def _check(got, want, mode, after):
    assert want["status"] == 0
    assert np.array_equal(got["U"], want["U"])
    assert np.array_equal(got["pos"], want["pos"])
    assert np.array_equal(got["missing"], want["missing"])
    assert np.array_equal(got["new_slot"], want["new_slot"])
    assert np.array_equal(after, want["slot_of"])
    if mode == gc.REORG_PACK:
        assert np.array_equal(got["pranges"], want["pranges"])
        assert np.array_equal(got["pi_begin"], want["pi_begin"])
    else:
        assert np.array_equal(got["ilist"], want["ilist"])


@pytest.mark.parametrize("mode", [gc.REORG_PACK, gc.REORG_INDIRECT])
@pytest.mark.parametrize("fill", [0.0, 0.95])
def test_wide_free_scan_maps_bit_exact(ctx, mode, fill):
    # a union of 2^18 ids in runs of 64, half of it resident at random slots; with fill 0.95 the pool
    # also holds other ids in 95 % of its slots, so the free slots the request takes are spread over
    # every wide block
    torch = torch_cuda()
    print(f"[gpu] wide free scan mode={mode} fill={fill}", flush=True)
    rng = np.random.default_rng(71 + int(fill * 100))
    tasks, union = _runs(rng, 4096)
    res_ids = np.sort(rng.choice(union, size=union.size // 2, replace=False))
    n_fill = int(fill * N) - res_ids.size if fill > 0 else 0
    others = np.setdiff1d(np.arange(N), union)
    fill_ids = np.sort(rng.choice(others, size=max(n_fill, 0), replace=False)) if n_fill > 0 else np.zeros(0, np.int64)
    ids = np.concatenate([res_ids, fill_ids]).astype(np.int32)
    slots = rng.choice(N, size=ids.size, replace=False).astype(np.int32)
    dev = torch.device("cuda")
    src = torch.rand((N, 4), device=dev)
    pool = gc.Pool(ctx, N, N)
    pool.set_source(src)
    pool.place(torch.from_numpy(ids).to(dev), torch.from_numpy(slots).to(dev))
    before = pool.query()
    want = O.maps(tasks, N, N, before, mode)
    b = gc.Batch(ctx, gc.KIND_GRAV, N)
    b.submit(gc.tasks_from_csr(tasks["i_begin"], tasks["i_count"], tasks["j_first"], tasks["j_nr"]),
             tasks["ranges"])
    b.commit()
    for call in range(2):
        b.reorganize(pool, mode)
        got = b.maps()
        _check(got, want, mode, pool.query())
        pool.evict_staged(b)
        assert np.array_equal(pool.query(), before), call
    b.status()
    b.destroy()
    pool.destroy()
