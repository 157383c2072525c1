"""FP64 checker for the combined force path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The device library never calls it and
shares no code with it; the only common module is ``workloads`` (seeded
inputs, no force arithmetic).

Every routine promotes the FP32 values the device consumes to FP64 and sums
serially per target in FP64; see ``oracle.c`` for the formulas.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

I32 = ctypes.POINTER(ctypes.c_int32)
I64 = ctypes.POINTER(ctypes.c_int64)
F32 = ctypes.POINTER(ctypes.c_float)
F64 = ctypes.POINTER(ctypes.c_double)

REDUNDANT, INDIRECT, SORTED, PACK = 0, 1, 2, 3


def build_native(force: bool = True) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_native(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.or_grav_lists.argtypes = [i32, I32, I32, I32, I32, I32, I32, I32, I32, F64, F64, F64, i32, dbl, dbl, F64, F64]
    lib.or_grav_brute.argtypes = [i64, F64, F64, dbl, dbl, F64, F64]
    lib.or_node_acc_points.argtypes = [i64, F64, F64, i32, dbl, dbl, F64]
    lib.or_node_moments.argtypes = [i32, I32, F64, F64, F64]
    lib.or_union_insert.restype = i64
    lib.or_union_insert.argtypes = [i32, I32, I32, I32, I32, I32, I32]
    lib.or_maps.restype = i32
    lib.or_maps.argtypes = [i32, I32, I32, I32, I32, I32, i32, i32, i32, I32, i32, I32, I32, I32, I32, I32, I32,
                            I32, I32, I64]
    lib.or_lj_tasks.argtypes = [i32, I32, I32, I32, I32, I32, F32, F32, i64, i32, F64, F64, F64, dbl, F64, F64, I64]
    lib.or_lj_brute.argtypes = [i64, F32, F64, F64, F64, F64, dbl, F64, F64]
    lib.or_ewald.argtypes = [i64, F64, dbl, dbl, dbl, F64, F64, dbl, i32, i32, F64, F64]
    lib.or_bh_walk.argtypes = [i32, I32, I32, F64, F64, F32, i32, I32, dbl, I32, I32, I64, I64, I32, I32]
    lib.or_vjp_grav_mono.argtypes = [i32, I32, I32, I32, I32, I32, I32, I32, I32, i32, I32, F64, F64, F64, dbl, dbl,
                                     F64, i64, F64, F64]
    lib.or_vjp_grav.argtypes = [i32, I32, I32, I32, I32, I32, I32, I32, I32, i32, I32, F64, F64, F64, i32, dbl, dbl,
                                F64, i64, F64, F64]
    lib.or_vjp_lj.argtypes = [i32, I32, I32, I32, I32, I32, F32, F32, F64, F64, i64, i32, F64, F64, dbl, F64, F64,
                              F64, F64, F64]
    lib.or_lj_energy_at.restype = dbl
    lib.or_lj_energy_at.argtypes = [i32, I32, I32, I32, I32, I32, F32, F32, F64, F64, F64, dbl]
    lib.or_lj_tasks_at.argtypes = [i32, I32, I32, I32, I32, I32, F32, F32, F64, F64, i64, F64, F64, dbl, F64]
    _lib = lib
    return lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a, t):
    return a.ctypes.data_as(t)


def _i(a):
    return _c(a, np.int32)


def _d(a):
    return _c(a, np.float64)


def moments_from_nodes32(nodes32: np.ndarray) -> np.ndarray:
    """FP32 node records (com, M, S6, T, pad) promoted to FP64 moments (com, M, S6)."""
    return _d(nodes32[:, :10])


# ---------------------------------------------------------------- gravity

def grav_lists(tasks: dict, pos, mass, mom, order: int, G: float = 1.0, eps: float = 0.01, n: int | None = None,
               potential: bool = False):
    """Acceleration (n x 3, FP64) of every target id over its task's lists; rows of ids not targeted stay NaN.
    With potential: (acc, pot) with pot (n) the potential of the same terms."""
    lib = _load()
    pos, mass, mom = _d(pos), _d(mass), _d(mom)
    n = pos.shape[0] if n is None else n
    acc = np.full((n, 3), np.nan)
    pot = np.full(n, np.nan) if potential else None
    t = {k: _i(v) for k, v in tasks.items()}
    lib.or_grav_lists(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32), _p(t["n_first"], I32),
                      _p(t["n_count"], I32), _p(t["j_first"], I32), _p(t["j_nr"], I32), _p(t["node_idx"], I32),
                      _p(t["ranges"], I32), _p(pos, F64), _p(mass, F64), _p(mom, F64), int(order), G, eps,
                      _p(acc, F64), _p(pot, F64) if potential else None)
    return (acc, pot) if potential else acc


def grav_brute(pos, mass, G: float = 1.0, eps: float = 0.01, potential: bool = False):
    lib = _load()
    pos, mass = _d(pos), _d(mass)
    n = pos.shape[0]
    acc = np.empty((n, 3))
    pot = np.empty(n) if potential else None
    lib.or_grav_brute(n, _p(pos, F64), _p(mass, F64), G, eps, _p(acc, F64), _p(pot, F64) if potential else None)
    return (acc, pot) if potential else acc


def node_acc_points(x, mom, order: int, G: float = 1.0, eps: float = 0.0):
    lib = _load()
    x, mom = _d(x), _d(mom)
    acc = np.empty_like(x)
    lib.or_node_acc_points(x.shape[0], _p(x, F64), _p(mom, F64), int(order), G, eps, _p(acc, F64))
    return acc


def node_moments(node_range, pos, mass):
    lib = _load()
    node_range, pos, mass = _i(node_range), _d(pos), _d(mass)
    mom = np.empty((node_range.shape[0], 10))
    lib.or_node_moments(node_range.shape[0], _p(node_range, I32), _p(pos, F64), _p(mass, F64), _p(mom, F64))
    return mom


def workload_tasks(w) -> dict:
    return dict(i_begin=w.i_begin, i_count=w.i_count, n_first=w.n_first, n_count=w.n_count, j_first=w.j_first,
                j_nr=w.j_nr, node_idx=w.node_idx, ranges=w.ranges)


def grav_workload(w, order: int, G: float = 1.0, eps: float = 0.01, tasks: dict | None = None,
                  potential: bool = False):
    """Oracle accelerations (and with potential, (acc, pot)) for a GravWorkload's FP32 records and FP32
    node table (promoted)."""
    rec = w.rec.astype(np.float64)
    return grav_lists(tasks if tasks is not None else workload_tasks(w), rec[:, :3], rec[:, 3],
                      moments_from_nodes32(w.nodes), order, G, eps, potential=potential)


# ---------------------------------------------------------------- maps

def union_insert(tasks: dict, n_ids: int) -> np.ndarray:
    lib = _load()
    t = {k: _i(v) for k, v in tasks.items()}
    U = np.empty(max(n_ids, 1), np.int32)
    nu = lib.or_union_insert(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32),
                             _p(t["j_first"], I32), _p(t["j_nr"], I32), _p(t["ranges"], I32), _p(U, I32))
    return U[:nu].copy()


def maps(tasks: dict, n_ids: int, capacity: int, slot_of, mode: int) -> dict:
    """All reorganisation maps of one combined request against pool state `slot_of` (not modified)."""
    lib = _load()
    t = {k: _i(v) for k, v in tasks.items()}
    T = int(t["i_begin"].shape[0])
    nr = int(t["ranges"].shape[0]) if t["ranges"].ndim == 2 else int(t["ranges"].size // 2)
    so = _i(slot_of).copy()
    U = np.empty(max(n_ids, 1), np.int32)
    pos = np.empty(max(n_ids, 1), np.int32)
    missing = np.empty(max(n_ids, 1), np.int32)
    new_slot = np.empty(max(n_ids, 1), np.int32)
    pranges = np.empty((max(nr, 1), 2), np.int32)
    pib = np.empty(max(T, 1), np.int32)
    ni = int(np.sum(t["i_count"], dtype=np.int64))
    rr = t["ranges"].reshape(-1, 2)
    nj = int(np.sum(rr[:, 1], dtype=np.int64))
    ilist = np.empty(max(ni, 1), np.int32)
    jlist = np.empty(max(nj, 1), np.int32)
    counts = np.zeros(2, np.int64)
    rc = lib.or_maps(T, _p(t["i_begin"], I32), _p(t["i_count"], I32), _p(t["j_first"], I32), _p(t["j_nr"], I32),
                     _p(t["ranges"], I32), nr, n_ids, capacity, _p(so, I32), int(mode), _p(U, I32), _p(pos, I32),
                     _p(missing, I32), _p(new_slot, I32), _p(pranges, I32), _p(pib, I32), _p(ilist, I32),
                     _p(jlist, I32), _p(counts, I64))
    nu, nm = int(counts[0]), int(counts[1])
    out = dict(status=int(rc), U=U[:nu].copy(), pos=pos[:n_ids].copy(), missing=missing[:nm].copy(), slot_of=so)
    if rc != 0:
        return out
    if mode in (REDUNDANT, PACK):
        out.update(pranges=pranges[:nr].copy(), pi_begin=pib[:T].copy())
        if mode == PACK:
            out["new_slot"] = new_slot[:nm].copy()
    else:
        out.update(new_slot=new_slot[:nm].copy(), ilist=ilist[:ni].copy(), jlist=jlist[:nj].copy())
    return out


# ---------------------------------------------------------------- Lennard-Jones

def lj_tasks(w, potential: bool = False, tasks: dict | None = None):
    lib = _load()
    t = tasks if tasks is not None else dict(i_begin=w.i_begin, i_count=w.i_count, j_begin=w.j_begin,
                                              j_count=w.j_count, self_flag=w.self_flag, shift=w.shift)
    ti = {k: _i(t[k]) for k in ("i_begin", "i_count", "j_begin", "j_count", "self_flag")}
    sh = _c(t["shift"], np.float32)
    rec = _c(w.rec, np.float32)
    n = rec.shape[0]
    acc = np.empty((n, 3))
    pot = np.zeros(n) if potential else None
    cnt = np.zeros(1, np.int64)
    lib.or_lj_tasks(int(ti["i_begin"].shape[0]), _p(ti["i_begin"], I32), _p(ti["i_count"], I32),
                    _p(ti["j_begin"], I32), _p(ti["j_count"], I32), _p(ti["self_flag"], I32), _p(sh, F32),
                    _p(rec, F32), n, int(w.eps_t.size), _p(_d(w.eps_t), F64), _p(_d(w.sig_t), F64),
                    _p(_d(w.mass_t), F64), w.rcut, _p(acc, F64), _p(pot, F64) if potential else None, _p(cnt, I64))
    return (acc, pot, int(cnt[0])) if potential else acc


def ewald(pos, L: float, G: float, M: float, com, alpha: float, nrep: int, hmax2: int, potential: bool = False,
          S=None):
    """Ewald correction of periodic gravity at each position (see oracle.c): acc (n x 3) [, phi (n)].
    S: the box's second moment about com (xx, yy, zz, xy, xz, yz), or None for the monopole alone."""
    lib = _load()
    pos = _d(pos)
    n = pos.shape[0]
    acc = np.empty((n, 3))
    pot = np.empty(n) if potential else None
    Sd = None if S is None else _d(np.asarray(S, dtype=np.float64).reshape(6))
    lib.or_ewald(n, _p(pos, F64), float(L), float(G), float(M), _p(_d(com), F64), _p(Sd, F64) if S is not None else None,
                 float(alpha), int(nrep), int(hmax2), _p(acc, F64), _p(pot, F64) if potential else None)
    return (acc, pot) if potential else acc


def lj_brute(w, potential: bool = False):
    lib = _load()
    rec = _c(w.rec, np.float32)
    n = rec.shape[0]
    acc = np.empty((n, 3))
    pot = np.empty(n) if potential else None
    lib.or_lj_brute(n, _p(rec, F32), _p(_d(w.L), F64), _p(_d(w.eps_t), F64), _p(_d(w.sig_t), F64),
                    _p(_d(w.mass_t), F64), w.rcut, _p(acc, F64), _p(pot, F64) if potential else None)
    return (acc, pot) if potential else acc


# ---------------------------------------------------------------- adjoints

def vjp_grav_mono(w, g, G: float = 1.0, eps: float = 0.01, pos=None, mass=None, mom=None):
    """(gpos n x 3, gmass n) of L = sum g_i . a_i over w's lists (direct + monopole), lists frozen."""
    lib = _load()
    rec = w.rec.astype(np.float64)
    pos = _d(rec[:, :3] if pos is None else pos)
    mass = _d(rec[:, 3] if mass is None else mass)
    mom = _d(moments_from_nodes32(w.nodes) if mom is None else mom)
    t = {k: _i(v) for k, v in workload_tasks(w).items()}
    nr = _i(w.node_range)
    g = _d(g)
    n = pos.shape[0]
    gpos = np.empty((n, 3))
    gmass = np.empty(n)
    lib.or_vjp_grav_mono(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32),
                         _p(t["n_first"], I32), _p(t["n_count"], I32), _p(t["j_first"], I32), _p(t["j_nr"], I32),
                         _p(t["node_idx"], I32), _p(t["ranges"], I32), int(nr.shape[0]), _p(nr, I32), _p(pos, F64),
                         _p(mass, F64), _p(mom, F64), G, eps, _p(g, F64), n, _p(gpos, F64), _p(gmass, F64))
    return gpos, gmass


def vjp_grav(w, g, order: int, G: float = 1.0, eps: float = 0.01, pos=None, mass=None, mom=None):
    """(gpos n x 3, gmass n) of L = sum g_i . a_i over w's lists with node terms of `order`, lists frozen."""
    lib = _load()
    rec = w.rec.astype(np.float64)
    pos = _d(rec[:, :3] if pos is None else pos)
    mass = _d(rec[:, 3] if mass is None else mass)
    mom = _d(moments_from_nodes32(w.nodes) if mom is None else mom)
    t = {k: _i(v) for k, v in workload_tasks(w).items()}
    nr = _i(w.node_range)
    g = _d(g)
    n = pos.shape[0]
    gpos = np.empty((n, 3))
    gmass = np.empty(n)
    lib.or_vjp_grav(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32),
                    _p(t["n_first"], I32), _p(t["n_count"], I32), _p(t["j_first"], I32), _p(t["j_nr"], I32),
                    _p(t["node_idx"], I32), _p(t["ranges"], I32), int(nr.shape[0]), _p(nr, I32), _p(pos, F64),
                    _p(mass, F64), _p(mom, F64), int(order), G, eps, _p(g, F64), n, _p(gpos, F64), _p(gmass, F64))
    return gpos, gmass


def _lj_t(w):
    return {k: _i(getattr(w, k)) for k in ("i_begin", "i_count", "j_begin", "j_count", "self_flag")}


def vjp_lj(w, g, pos=None, mass=None, eps_t=None, sig_t=None):
    """(gpos, gmass per atom, geps_t, gsig_t) of L = sum g_i . a_i over w's cell-pair tasks."""
    lib = _load()
    t = _lj_t(w)
    rec = _c(w.rec, np.float32)
    n = rec.shape[0]
    pos = _d(rec[:, :3].astype(np.float64) if pos is None else pos)
    mass = _d(w.mass_t[rec[:, 3].astype(np.int64)].astype(np.float64) if mass is None else mass)
    eps_t = _d(w.eps_t if eps_t is None else eps_t)
    sig_t = _d(w.sig_t if sig_t is None else sig_t)
    g = _d(g)
    nt = int(eps_t.size)
    gpos, gmass, ge, gs = np.empty((n, 3)), np.empty(n), np.empty(nt), np.empty(nt)
    lib.or_vjp_lj(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32), _p(t["j_begin"], I32),
                  _p(t["j_count"], I32), _p(t["self_flag"], I32), _p(_c(w.shift, np.float32), F32), _p(rec, F32),
                  _p(pos, F64), _p(mass, F64), n, nt, _p(eps_t, F64), _p(sig_t, F64), w.rcut, _p(g, F64),
                  _p(gpos, F64), _p(gmass, F64), _p(ge, F64), _p(gs, F64))
    return gpos, gmass, ge, gs


def lj_energy_at(w, pos, eps_t=None, sig_t=None) -> float:
    """Total (unshifted) LJ potential energy at FP64 positions, w's cutoff decisions frozen."""
    lib = _load()
    t = _lj_t(w)
    rec = _c(w.rec, np.float32)
    pos = _d(pos)
    eps_t = _d(w.eps_t if eps_t is None else eps_t)
    sig_t = _d(w.sig_t if sig_t is None else sig_t)
    return float(lib.or_lj_energy_at(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32),
                                      _p(t["j_begin"], I32), _p(t["j_count"], I32), _p(t["self_flag"], I32),
                                      _p(_c(w.shift, np.float32), F32), _p(rec, F32), _p(pos, F64),
                                      _p(eps_t, F64), _p(sig_t, F64), w.rcut))


def lj_at(w, pos, mass, eps_t, sig_t):
    """LJ accelerations at FP64 positions/masses/parameters with w's cutoff decisions frozen."""
    lib = _load()
    t = _lj_t(w)
    rec = _c(w.rec, np.float32)
    n = rec.shape[0]
    pos, mass, eps_t, sig_t = _d(pos), _d(mass), _d(eps_t), _d(sig_t)
    acc = np.empty((n, 3))
    lib.or_lj_tasks_at(int(t["i_begin"].shape[0]), _p(t["i_begin"], I32), _p(t["i_count"], I32),
                       _p(t["j_begin"], I32), _p(t["j_count"], I32), _p(t["self_flag"], I32),
                       _p(_c(w.shift, np.float32), F32), _p(rec, F32), _p(pos, F64), _p(mass, F64), n,
                       _p(eps_t, F64), _p(sig_t, F64), w.rcut, _p(acc, F64))
    return acc


# ---------------------------------------------------------------- metrics

def per_task_rel_l2(acc_test, acc_ref, i_begin, i_count, floor_frac: float = 0.0):
    """Per task ||a_test - a_ref||_2 / ||a_ref||_2 over its 3*i_count components.

    With floor_frac > 0, a task whose reference norm is below floor_frac x the median task norm is
    measured against floor_frac x median instead (absolute guard for near-zero reference forces)."""
    acc_test = np.asarray(acc_test, np.float64)
    acc_ref = np.asarray(acc_ref, np.float64)
    idx = np.repeat(np.arange(len(i_begin)), i_count)
    ids = np.concatenate([np.arange(b, b + c) for b, c in zip(i_begin, i_count)]) if len(i_begin) else np.zeros(0, int)
    err2 = np.bincount(idx, weights=np.sum((acc_test[ids] - acc_ref[ids]) ** 2, axis=1), minlength=len(i_begin))
    ref2 = np.bincount(idx, weights=np.sum(acc_ref[ids] ** 2, axis=1), minlength=len(i_begin))
    den = np.sqrt(ref2)
    if floor_frac > 0 and den.size:
        den = np.maximum(den, floor_frac * np.median(den))
    return np.sqrt(err2) / np.where(den > 0, den, 1.0)


# ---------------------------------------------------------------- interaction lists

def bh_walk(node_range, node_parent, node_side, node_com, rec, bucket_node, theta: float):
    """Barnes-Hut lists of each bucket (see oracle.c): (n_first (nb + 1), node_idx, r_first (nb + 1),
    ranges (n x 2)), in the walk's order."""
    lib = _load()
    nr = _c(node_range, np.int32)
    par = _c(node_parent, np.int32)
    side = _d(node_side)
    com = _d(node_com)
    rec = _c(rec, np.float32)
    bn = _c(bucket_node, np.int32)
    nn, nb = nr.shape[0], bn.shape[0]
    nc = np.zeros(max(nb, 1), np.int32)
    rc = np.zeros(max(nb, 1), np.int32)
    lib.or_bh_walk(nn, _p(nr, I32), _p(par, I32), _p(side, F64), _p(com, F64), _p(rec, F32), nb, _p(bn, I32),
                   float(theta), _p(nc, I32), _p(rc, I32), None, None, None, None)
    nf = np.concatenate([[0], np.cumsum(nc[:nb], dtype=np.int64)])
    rf = np.concatenate([[0], np.cumsum(rc[:nb], dtype=np.int64)])
    node_idx = np.zeros(max(int(nf[-1]), 1), np.int32)
    ranges = np.zeros((max(int(rf[-1]), 1), 2), np.int32)
    nf64, rf64 = _c(nf, np.int64), _c(rf, np.int64)
    lib.or_bh_walk(nn, _p(nr, I32), _p(par, I32), _p(side, F64), _p(com, F64), _p(rec, F32), nb, _p(bn, I32),
                   float(theta), None, None, _p(nf64, I64), _p(rf64, I64), _p(node_idx, I32), _p(ranges, I32))
    return nf.astype(np.int32), node_idx[:int(nf[-1])], rf.astype(np.int32), ranges[:int(rf[-1])]


def bh_walk_workload(w, theta: float | None = None):
    """bh_walk over a gravity workload's tree (theta defaults to the workload's)."""
    return bh_walk(w.node_range, w.node_parent, w.node_side, w.node_mom64[:, :3], w.rec, w.meta["leaf"],
                   w.theta if theta is None else theta)
