"""gc_tree_walk_noalloc (the list walk with its scratch in the library's fixed device array) against
gc_tree_walk: bit-exact lists on two calls in a row, the second with a smaller tree, and the refusal of a
tree larger than the fixed scratch."""
import ctypes

import numpy as np
import pytest

import paper_2008_05712_amd as gc
import workloads as W

pytestmark = pytest.mark.gpu


def _dev_args(w):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
            (w.node_range.astype(np.int32), w.node_mom64[:, :3], w.node_side, w.rec, w.meta["leaf"].astype(np.int32))]


def _cpu(t):
    return t.cpu().numpy()


def test_noalloc_walk_matches_the_allocating_walk():
    import torch
    ctx = gc.Context(0)
    for w in (W.nbody_plummer(), W.nbody_tiny()):  # the second call walks a smaller tree
        print(f"[gpu] no-allocation walk N={w.n} nodes={w.node_range.shape[0]}", flush=True)
        args = _dev_args(w)
        want = gc.tree_walk(ctx, *args, w.theta)
        got = gc.tree_walk(ctx, *args, w.theta, noalloc=True)
        torch.cuda.synchronize()
        for a, b in zip(want, got):
            assert a.shape == b.shape
            assert np.array_equal(_cpu(a), _cpu(b))
        # totals and offsets describe the lists the oracle's walk defines (node and range counts)
        assert int(_cpu(got[0])[-1]) == got[1].numel() and int(_cpu(got[2])[-1]) == got[3].shape[0]
    ctx.close()


def test_noalloc_walk_refuses_a_tree_beyond_its_scratch():
    ctx = gc.Context(0)
    w = W.nbody_tiny()
    args = _dev_args(w)
    totals = (ctypes.c_int64 * 2)()
    n_first = args[0].new_empty(int(args[4].numel()) + 1)
    st = gc.lib().gc_tree_walk_noalloc(ctx.h, (1 << 21) + 1, args[0].data_ptr(), args[1].data_ptr(),
                                       args[2].data_ptr(), args[3].data_ptr(), w.n, int(args[4].numel()),
                                       args[4].data_ptr(), float(w.theta), n_first.data_ptr(), n_first.data_ptr(),
                                       None, 0, None, 0, totals, None)
    assert st == gc.GC_E_INVAL
    assert b"fixed scratch" in gc.lib().gc_last_error(ctx.h)
    ctx.close()
