"""Seeded synthetic inputs for the combined force path.

This module only prepares inputs: particle distributions, the octree and the
bucket interaction lists a Barnes-Hut walk produces (the work requests of the
N-body application, Sec. 4.1), Lennard-Jones cell-pair tasks (the compute
objects of the MD application, Sec. 4.2), arrival rounds and pool residency
fixtures (Sec. 3.1, Sec. 3.2).  It evaluates no forces and shares nothing with
the device library or the checker beyond the arrays it returns.

Random numbers come from numpy's PCG64 (``numpy.random.default_rng(seed)``).
The native part (tree build, walk, cell sort) is ``gen.c``, built into
``libworkloads.so`` beside this file by :func:`build_native`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libworkloads.so")
_lib = None

I32 = ctypes.POINTER(ctypes.c_int32)
F32 = ctypes.POINTER(ctypes.c_float)
F64 = ctypes.POINTER(ctypes.c_double)


def build_native(force: bool = True) -> str:
    """Compile gen.c into libworkloads.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build_native(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.wl_tree_build.restype = ctypes.c_void_p
    lib.wl_tree_build.argtypes = [ctypes.c_int64, F32, ctypes.c_int32]
    lib.wl_tree_free.argtypes = [ctypes.c_void_p]
    lib.wl_tree_nnodes.restype = ctypes.c_int32
    lib.wl_tree_nnodes.argtypes = [ctypes.c_void_p]
    lib.wl_tree_nleaves.restype = ctypes.c_int32
    lib.wl_tree_nleaves.argtypes = [ctypes.c_void_p]
    lib.wl_tree_export.argtypes = [ctypes.c_void_p, I32, F32, F32, I32, F64, I32, I32, F64]
    lib.wl_walk.restype = ctypes.c_void_p
    lib.wl_walk.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.wl_lists_sizes.argtypes = [ctypes.c_void_p, I32, I32, I32]
    lib.wl_lists_export.argtypes = [ctypes.c_void_p, I32, I32, I32, I32, I32]
    lib.wl_lists_free.argtypes = [ctypes.c_void_p]
    lib.wl_cells_dims.restype = ctypes.c_int32
    lib.wl_cells_dims.argtypes = [F64, ctypes.c_double, I32]
    lib.wl_cells_sort.argtypes = [ctypes.c_int64, F32, F64, I32, I32, I32]
    lib.wl_cells_tasks.argtypes = [F64, I32, I32, I32, F32]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


# --------------------------------------------------------------------------
# distributions
# --------------------------------------------------------------------------

def uniform_cube(n: int, seed: int) -> np.ndarray:
    """n particles uniform in [0,1)^3, equal masses 1/n; FP64 draws rounded to FP32 records (x, y, z, m)."""
    rng = np.random.default_rng(seed)
    rec = np.empty((n, 4), np.float32)
    rec[:, :3] = rng.random((n, 3))
    rec[:, 3] = np.float32(1.0 / n)
    return rec


def plummer(n: int, seed: int, a: float = 1.0, rmax: float = 10.0) -> np.ndarray:
    """Plummer sphere of scale radius a, cut at rmax (rejection), isotropic, masses 1/n.

    Radius by inverting the cumulative mass M(r) = r^3 / (r^2 + a^2)^{3/2}:
    r = a (X^{-2/3} - 1)^{-1/2} for X uniform in (0, 1).
    """
    rng = np.random.default_rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = n - out.shape[0]
        X = rng.random(m + m // 16 + 16)
        X = X[X > 0]
        r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        r = r[r <= rmax]
        u = rng.random((r.size, 2))
        cth = 2.0 * u[:, 0] - 1.0
        sth = np.sqrt(1.0 - cth * cth)
        ph = 2.0 * math.pi * u[:, 1]
        xyz = np.stack([r * sth * np.cos(ph), r * sth * np.sin(ph), r * cth], axis=1)
        out = np.concatenate([out, xyz])[:n]
    rec = np.empty((n, 4), np.float32)
    rec[:, :3] = out
    rec[:, 3] = np.float32(1.0 / n)
    return rec


def log_uniform_sizes(k: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=k))).astype(np.int64)


# --------------------------------------------------------------------------
# N-body: octree, walk, tasks
# --------------------------------------------------------------------------

@dataclass
class GravWorkload:
    """One N-body instance in relabelled (depth-first leaf) id order.

    rec        float32[N,4]   (x, y, z, m) by id
    perm       int32[N]       perm[id] = input index
    nodes      float32[NN,12] (com x y z, M, Sxx Syy Szz Sxy, Sxz Syz T, 0)
    node_range int32[NN,2]    (first id, count)
    node_parent int32[NN]     parent node (-1 root)
    node_side  float64[NN]    cube side
    tasks: i_begin, i_count, n_first, n_count, j_first, j_nr  int32[T]
    node_idx   int32[sum n_count]
    ranges     int32[sum j_nr, 2]  (first id, count)
    """
    rec: np.ndarray
    perm: np.ndarray
    nodes: np.ndarray
    node_range: np.ndarray
    node_parent: np.ndarray
    node_side: np.ndarray
    node_mom64: np.ndarray
    i_begin: np.ndarray
    i_count: np.ndarray
    n_first: np.ndarray
    n_count: np.ndarray
    j_first: np.ndarray
    j_nr: np.ndarray
    node_idx: np.ndarray
    ranges: np.ndarray
    theta: float
    bucket: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.rec.shape[0]

    @property
    def n_tasks(self) -> int:
        return self.i_begin.shape[0]

    def direct_counts(self) -> np.ndarray:
        """Direct j-particles per task (including the target itself)."""
        cs = np.concatenate([[0], np.cumsum(self.ranges[:, 1].astype(np.int64))])
        return cs[self.j_first + self.j_nr] - cs[self.j_first]

    def interactions(self) -> int:
        """Sum over tasks of i_count * (direct particles excluding self + nodes)."""
        return int(np.sum(self.i_count.astype(np.int64) * (self.direct_counts() - 1 + self.n_count)))

    def split_interactions(self):
        """(direct pair interactions excluding self, node interactions)."""
        ic = self.i_count.astype(np.int64)
        return int(np.sum(ic * (self.direct_counts() - 1))), int(np.sum(ic * self.n_count))


def build_grav(rec_in: np.ndarray, bucket: int, theta: float) -> GravWorkload:
    """Octree + Barnes-Hut walk over FP32 records (input order); returns relabelled arrays."""
    lib = _load()
    rec_in = np.ascontiguousarray(rec_in, np.float32)
    n = rec_in.shape[0]
    t = lib.wl_tree_build(n, _p(rec_in, F32), bucket)
    if not t:
        raise ValueError("tree build failed")
    try:
        nn = lib.wl_tree_nnodes(t)
        perm = np.empty(n, np.int32)
        rec = np.empty((n, 4), np.float32)
        nodes = np.empty((nn, 12), np.float32)
        node_range = np.empty((nn, 2), np.int32)
        geom = np.empty((nn, 4), np.float64)
        depth = np.empty(nn, np.int32)
        parent = np.empty(nn, np.int32)
        mom64 = np.empty((nn, 10), np.float64)
        lib.wl_tree_export(t, _p(perm, I32), _p(rec, F32), _p(nodes, F32), _p(node_range, I32),
                           _p(geom, F64), _p(depth, I32), _p(parent, I32), _p(mom64, F64))
        L = lib.wl_walk(t, float(theta))
        try:
            nb, nref, nrng = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            lib.wl_lists_sizes(L, ctypes.byref(nb), ctypes.byref(nref), ctypes.byref(nrng))
            nb, nref, nrng = nb.value, nref.value, nrng.value
            leaf = np.empty(nb, np.int32)
            nfirst = np.empty(nb + 1, np.int32)
            rfirst = np.empty(nb + 1, np.int32)
            node_idx = np.empty(max(nref, 1), np.int32)
            ranges = np.empty((max(nrng, 1), 2), np.int32)
            lib.wl_lists_export(L, _p(leaf, I32), _p(nfirst, I32), _p(rfirst, I32), _p(node_idx, I32), _p(ranges, I32))
        finally:
            lib.wl_lists_free(L)
    finally:
        lib.wl_tree_free(t)
    return GravWorkload(
        rec=rec, perm=perm, nodes=nodes, node_range=node_range, node_parent=parent,
        node_side=geom[:, 3].copy(), node_mom64=mom64,
        i_begin=node_range[leaf, 0].copy(), i_count=node_range[leaf, 1].copy(),
        n_first=nfirst[:-1].copy(), n_count=np.diff(nfirst).astype(np.int32),
        j_first=rfirst[:-1].copy(), j_nr=np.diff(rfirst).astype(np.int32),
        node_idx=node_idx[:nref], ranges=ranges[:nrng], theta=float(theta), bucket=int(bucket),
        meta={"leaf": leaf, "node_depth": depth, "node_geom": geom})


def concat_grav(ws: list[GravWorkload]) -> GravWorkload:
    """Independent instances in one id space: ids, node indices and lists are offset per instance."""
    id_off = np.cumsum([0] + [w.n for w in ws])
    nd_off = np.cumsum([0] + [w.nodes.shape[0] for w in ws])
    nr_off = np.cumsum([0] + [w.node_idx.shape[0] for w in ws])
    rg_off = np.cumsum([0] + [w.ranges.shape[0] for w in ws])
    cat = np.concatenate
    parent = cat([np.where(w.node_parent >= 0, w.node_parent + nd_off[k], -1) for k, w in enumerate(ws)]).astype(np.int32)
    out = GravWorkload(
        rec=cat([w.rec for w in ws]), perm=cat([w.perm + id_off[k] for k, w in enumerate(ws)]).astype(np.int32),
        nodes=cat([w.nodes for w in ws]),
        node_range=cat([w.node_range + np.array([id_off[k], 0]) for k, w in enumerate(ws)]).astype(np.int32),
        node_parent=parent, node_side=cat([w.node_side for w in ws]), node_mom64=cat([w.node_mom64 for w in ws]),
        i_begin=cat([w.i_begin + id_off[k] for k, w in enumerate(ws)]).astype(np.int32),
        i_count=cat([w.i_count for w in ws]),
        n_first=cat([w.n_first + nr_off[k] for k, w in enumerate(ws)]).astype(np.int32),
        n_count=cat([w.n_count for w in ws]),
        j_first=cat([w.j_first + rg_off[k] for k, w in enumerate(ws)]).astype(np.int32),
        j_nr=cat([w.j_nr for w in ws]),
        node_idx=cat([w.node_idx + nd_off[k] for k, w in enumerate(ws)]).astype(np.int32),
        ranges=cat([w.ranges + np.array([id_off[k], 0]) for k, w in enumerate(ws)]).astype(np.int32),
        theta=ws[0].theta, bucket=ws[0].bucket,
        meta={"instance_of_task": cat([np.full(w.n_tasks, k, np.int32) for k, w in enumerate(ws)]),
              "id_offset": id_off, "node_offset": nd_off})
    return out


def task_subset(w: GravWorkload, sel: np.ndarray) -> dict:
    """Tasks `sel` (indices) as a self-contained CSR batch (lists re-based to the subset)."""
    sel = np.asarray(sel, np.int64)
    nc = w.n_count[sel].astype(np.int64)
    jn = w.j_nr[sel].astype(np.int64)
    n_first = np.concatenate([[0], np.cumsum(nc)[:-1]]).astype(np.int32)
    j_first = np.concatenate([[0], np.cumsum(jn)[:-1]]).astype(np.int32)
    node_idx = np.concatenate([w.node_idx[w.n_first[t]:w.n_first[t] + w.n_count[t]] for t in sel]) if sel.size else np.zeros(0, np.int32)
    ranges = np.concatenate([w.ranges[w.j_first[t]:w.j_first[t] + w.j_nr[t]] for t in sel]) if sel.size else np.zeros((0, 2), np.int32)
    return dict(i_begin=w.i_begin[sel].astype(np.int32), i_count=w.i_count[sel].astype(np.int32),
                n_first=n_first, n_count=w.n_count[sel].astype(np.int32), j_first=j_first,
                j_nr=w.j_nr[sel].astype(np.int32), node_idx=node_idx.astype(np.int32),
                ranges=np.ascontiguousarray(ranges, np.int32).reshape(-1, 2))


def poisson_rounds(n_tasks: int, mean: float, seed: int, n_rounds: int | None = None) -> list[np.ndarray]:
    """Consecutive task rounds (tree order) of Poisson(mean) size (at least 1).  Without n_rounds: rounds
    until every task is covered once.  With n_rounds: exactly that many, wrapping from the last task to
    the first (a round that wraps holds the tail and then the head of the order); the first rounds are
    the same as without it."""
    rng = np.random.default_rng(seed)
    out, t = [], 0
    if n_rounds is None:
        while t < n_tasks:
            k = max(1, int(rng.poisson(mean)))
            out.append(np.arange(t, min(n_tasks, t + k), dtype=np.int64))
            t += k
        return out
    for _ in range(n_rounds):
        k = min(max(1, int(rng.poisson(mean))), n_tasks)
        out.append((t + np.arange(k, dtype=np.int64)) % n_tasks)
        t = (t + k) % n_tasks
    return out


def batch_union(batch: dict) -> np.ndarray:
    """Sorted unique ids over all i- and j-ranges of a batch."""
    parts = [np.arange(b, b + c) for b, c in zip(batch["i_begin"], batch["i_count"])]
    parts += [np.arange(b, b + c) for b, c in batch["ranges"]]
    return np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)


def residency(union: np.ndarray, capacity: int, frac: float, seed: int):
    """floor(frac * |U|) ids of U chosen uniformly, placed at distinct uniform random slots in [0, capacity)."""
    rng = np.random.default_rng(seed)
    k = int(math.floor(frac * union.size))
    ids = np.sort(rng.choice(union, size=k, replace=False)).astype(np.int32)
    slots = rng.choice(capacity, size=k, replace=False).astype(np.int32)
    return ids, slots


# --------------------------------------------------------------------------
# Lennard-Jones: lattice, cells, cell-pair tasks
# --------------------------------------------------------------------------

@dataclass
class LJWorkload:
    """Atoms in cell-sorted id order: rec float32[N,4] = (x, y, z, type), box L (FP64, FP32-exact).

    tasks: i_begin, i_count, j_begin, j_count, self_flag int32[T]; shift float32[T,3]
    """
    rec: np.ndarray
    perm: np.ndarray
    L: np.ndarray
    rcut: float
    ncell: np.ndarray
    cell_start: np.ndarray
    i_begin: np.ndarray
    i_count: np.ndarray
    j_begin: np.ndarray
    j_count: np.ndarray
    self_flag: np.ndarray
    shift: np.ndarray
    eps_t: np.ndarray
    sig_t: np.ndarray
    mass_t: np.ndarray
    vel: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.rec.shape[0]

    @property
    def n_tasks(self) -> int:
        return self.i_begin.shape[0]

    def candidates(self) -> int:
        ic = self.i_count.astype(np.int64)
        jc = self.j_count.astype(np.int64)
        return int(np.sum(np.where(self.self_flag != 0, ic * (ic - 1) // 2, ic * jc)))


def wrap_box(xyz: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Wrap FP32 positions into [0, L) per dimension (FP32 result)."""
    x = np.mod(xyz.astype(np.float64), L).astype(np.float32)
    Lf = L.astype(np.float32)
    x = np.where(x >= Lf, x - Lf, x)
    return np.where(x < 0, np.float32(0), x).astype(np.float32)


def build_lj(xyz: np.ndarray, types: np.ndarray, L, rcut: float, eps_t, sig_t, mass_t, vel=None) -> LJWorkload:
    lib = _load()
    L = np.asarray(L, np.float64)
    L = L.astype(np.float32).astype(np.float64)  # box lengths exactly representable in FP32
    n = xyz.shape[0]
    rec_in = np.empty((n, 4), np.float32)
    rec_in[:, :3] = wrap_box(np.asarray(xyz), L)
    rec_in[:, 3] = np.asarray(types, np.float32)
    ncell = np.empty(3, np.int32)
    if lib.wl_cells_dims(_p(L, F64), float(rcut), _p(ncell, I32)) != 0:
        raise ValueError("box must hold at least 3 cells of side >= r_cut per dimension")
    nc = int(np.prod(ncell.astype(np.int64)))
    perm = np.empty(n, np.int32)
    cell_start = np.empty(nc + 1, np.int32)
    lib.wl_cells_sort(n, _p(rec_in, F32), _p(L, F64), _p(ncell, I32), _p(perm, I32), _p(cell_start, I32))
    rec = rec_in[perm]
    it = np.empty((14 * nc, 5), np.int32)
    sh = np.empty((14 * nc, 3), np.float32)
    lib.wl_cells_tasks(_p(L, F64), _p(ncell, I32), _p(cell_start, I32), _p(it, I32), _p(sh, F32))
    return LJWorkload(rec=rec, perm=perm, L=L, rcut=float(rcut), ncell=ncell, cell_start=cell_start,
                      i_begin=it[:, 0].copy(), i_count=it[:, 1].copy(), j_begin=it[:, 2].copy(),
                      j_count=it[:, 3].copy(), self_flag=it[:, 4].copy(), shift=sh,
                      eps_t=np.asarray(eps_t, np.float32), sig_t=np.asarray(sig_t, np.float32),
                      mass_t=np.asarray(mass_t, np.float32), vel=None if vel is None else np.asarray(vel)[perm])


def fcc_modulated(nx: int, ny: int, nz: int, rho: float, n_target: int, seed: int, jitter: float = 0.05,
                  temperature: float = 1.0):
    """FCC lattice of nx*ny*nz unit cells at reduced density rho; seeded deletion of sites from the
    half-box x < Lx/2 down to n_target atoms in total; Gaussian jitter (sd `jitter`); Maxwell velocities
    at `temperature` (COM drift removed, rescaled exactly).  Returns (xyz float64[N,3], vel, L)."""
    rng = np.random.default_rng(seed)
    a = (4.0 / rho) ** (1.0 / 3.0)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    sites = ((g[:, None, :] + basis[None, :, :]).reshape(-1, 3)) * a
    L = np.array([nx * a, ny * a, nz * a])
    n_del = sites.shape[0] - n_target
    if n_del < 0:
        raise ValueError("n_target exceeds the lattice")
    left = np.nonzero(sites[:, 0] < L[0] / 2)[0]
    if n_del > left.size:
        raise ValueError("cannot delete that many sites from the half-box")
    drop = rng.choice(left, size=n_del, replace=False)
    keep = np.ones(sites.shape[0], bool)
    keep[drop] = False
    xyz = sites[keep] + rng.normal(0.0, jitter, size=(n_target, 3))
    v = rng.normal(0.0, 1.0, size=(n_target, 3))
    v -= v.mean(axis=0)
    v *= math.sqrt(3.0 * (n_target - 1) * temperature / np.sum(v * v))
    return xyz, v, L


def simple_cubic(n_side: int, rho: float, seed: int, jitter: float = 0.05):
    rng = np.random.default_rng(seed)
    a = (1.0 / rho) ** (1.0 / 3.0)
    g = np.stack(np.meshgrid(*(np.arange(n_side),) * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    xyz = (g + 0.5) * a + rng.normal(0.0, jitter, size=g.shape)
    L = np.full(3, n_side * a)
    return xyz, L


def two_types(n: int, seed: int) -> np.ndarray:
    """Half type 0, half type 1, seeded shuffle."""
    rng = np.random.default_rng(seed)
    t = np.zeros(n, np.int32)
    t[n // 2:] = 1
    rng.shuffle(t)
    return t


# --------------------------------------------------------------------------
# named configurations
# --------------------------------------------------------------------------

def nbody_tiny(seed: int = 1001, n: int = 4096, bucket: int = 16, theta: float = 0.7) -> GravWorkload:
    """4,096 particles uniform in the unit cube, masses 1/N, bucket 16, theta 0.7, monopole."""
    w = build_grav(uniform_cube(n, seed), bucket, theta)
    w.meta.update(config="nbody-uniform-4096", seed=seed)
    return w


def nbody_plummer(n: int = 262144, seed: int = 1002, bucket: int = 32, theta: float = 0.7) -> GravWorkload:
    """Plummer sphere (a = 1, cut at 10a), masses 1/N, bucket 32, theta 0.7, monopole + quadrupole."""
    w = build_grav(plummer(n, seed), bucket, theta)
    w.meta.update(config=f"nbody-plummer-{n}", seed=seed)
    return w


def nbody_instances(k: int = 64, lo: int = 2048, hi: int = 262144, seed: int = 4000, bucket: int = 32,
                    theta: float = 0.7) -> GravWorkload:
    sizes = log_uniform_sizes(k, lo, hi, seed)
    ws = [build_grav(plummer(int(s), seed + 1 + i), bucket, theta) for i, s in enumerate(sizes)]
    w = concat_grav(ws)
    w.meta.update(config=f"nbody-plummer-x{k}", sizes=sizes)
    return w


LJ_TWO_TYPES = dict(eps_t=[1.0, 0.5], sig_t=[1.0, 0.88], mass_t=[1.0, 1.0])


def lj_fcc(seed: int = 1003, nx: int = 75, ny: int = 64, nz: int = 64, n_target: int = 1048576,
           rho: float = 0.8442, rcut: float = 2.5, two_type: bool = False) -> LJWorkload:
    """FCC at reduced density 0.8442 with a seeded half-box thinned to ~0.6, 0.05 sigma jitter,
    Maxwell velocities at T = 1; one type (eps = sigma = m = 1) or the two-type mixture."""
    xyz, v, L = fcc_modulated(nx, ny, nz, rho, n_target, seed)
    if two_type:
        types = two_types(xyz.shape[0], seed + 7)
        prm = LJ_TWO_TYPES
    else:
        types = np.zeros(xyz.shape[0], np.int32)
        prm = dict(eps_t=[1.0], sig_t=[1.0], mass_t=[1.0])
    w = build_lj(xyz, types, L, rcut, vel=v, **prm)
    w.meta.update(config=f"lj-fcc-{xyz.shape[0]}", seed=seed)
    return w


def lj_small(seed: int = 5003, n_side: int = 8, rho: float = 0.8442, rcut: float = 2.5) -> LJWorkload:
    """n_side^3 simple-cubic sites at rho with 0.05 sigma jitter, two types (FD-sized instance)."""
    xyz, L = simple_cubic(n_side, rho, seed)
    types = two_types(xyz.shape[0], seed + 7)
    w = build_lj(xyz, types, L, rcut, **LJ_TWO_TYPES)
    w.meta.update(config=f"lj-sc-{xyz.shape[0]}", seed=seed)
    return w
