"""MI355X combined irregular-task force library: Python binding of the C ABI in include/gcharm.h.

Argument marshalling only: every step of the path (reorganisation, combined
force pass, adjoint) runs in the HIP kernels of ``libgcharm.so``.  PyTorch
supplies device memory and streams.  Importing works without the library;
the first call that needs it raises :class:`GcError` if ``libgcharm.so`` has
not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["GcError", "lib", "Context", "Pool", "Batch", "Graph", "Combiner", "ForceParams", "EwaldParams",
           "ewald_params", "Hybrid", "lj_forces_cpu", "tree_walk", "walk_tasks", "DEVICE_CPU", "DEVICE_GPU", "TASK_DTYPE",
           "REORG_REDUNDANT", "REORG_INDIRECT", "REORG_SORTED", "REORG_PACK", "REORG_NONE",
           "FORCE_GRAV_MONO", "FORCE_GRAV_QUAD", "FORCE_LJ", "KIND_GRAV", "KIND_LJ", "TASK_SELF",
           "FIXTURE_NONE", "FIXTURE_RESET_PLACE", "FIXTURE_EVICT_STAGED", "SCHED_TASKS", "SCHED_QUEUE", "SCHED_STEP",
           "SCHED_ROUNDS",
           "LIB_PATH", "EXPORTED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcharm.so")

GC_OK, GC_E_INVAL, GC_E_NOMEM, GC_E_FULL, GC_E_STATE, GC_E_HIP, GC_E_UNSUPPORTED = range(7)
KIND_GRAV, KIND_LJ = 0, 1
TASK_SELF = 1
REORG_REDUNDANT, REORG_INDIRECT, REORG_SORTED, REORG_PACK, REORG_NONE = 0, 1, 2, 3, 4
FORCE_GRAV_MONO, FORCE_GRAV_QUAD, FORCE_LJ = 1, 2, 3
FIXTURE_NONE, FIXTURE_RESET_PLACE, FIXTURE_EVICT_STAGED = 0, 1, 2
SCHED_TASKS, SCHED_QUEUE, SCHED_STEP, SCHED_ROUNDS = 0, 1, 2, 3

# gc_task: 7 int32 + 3 float32 = 40 bytes
TASK_DTYPE = np.dtype([("i_begin", "<i4"), ("i_count", "<i4"), ("j_first", "<i4"), ("j_nranges", "<i4"),
                       ("n_first", "<i4"), ("n_count", "<i4"), ("flags", "<i4"), ("shift", "<f4", (3,))])

EXPORTED = ["gc_version", "gc_init", "gc_finalize", "gc_last_error", "gc_debug_inject_error", "gc_debug_step_waits",
            "gc_batch_status", "gc_graph_status", "gc_pool_create", "gc_pool_destroy",
            "gc_pool_set_source", "gc_pool_set_host_source", "gc_pool_query_mirror", "gc_pool_place", "gc_pool_reset", "gc_pool_evict", "gc_pool_evict_staged",
            "gc_pool_query", "gc_pool_device_ptrs",
            "gc_batch_create", "gc_batch_destroy", "gc_batch_reset", "gc_submit_tasks", "gc_submit_tasks_device",
            "gc_walk_tasks", "gc_batch_commit",
            "gc_batch_sizes", "gc_reorganize", "gc_batch_maps", "gc_launch_combined", "gc_zero_f32", "gc_backward",
            "gc_graph_capture", "gc_graph_launch", "gc_graph_destroy", "gc_autotune", "gc_occupancy", "gc_lj_count_pairs",
            "gc_launch_ewald", "gc_hybrid_create", "gc_hybrid_destroy", "gc_hybrid_record", "gc_hybrid_split",
            "gc_hybrid_state", "gc_lj_forces_cpu", "gc_combiner_create", "gc_combiner_destroy", "gc_combiner_arrive", "gc_combiner_poll", "gc_combiner_state",
            "gc_tree_walk", "gc_tree_walk_noalloc"]


class EwaldParams(ctypes.Structure):
    """gc_ewald_params: box side, G, total mass, centre of mass, alpha (0: 2 / L), images, |h|^2 bound,
    second moment about the centre of mass (xx, yy, zz, xy, xz, yz; zeros: monopole only)."""
    _fields_ = [("L", ctypes.c_float), ("G", ctypes.c_float), ("M", ctypes.c_float), ("com", ctypes.c_float * 3),
                ("alpha", ctypes.c_float), ("nrep", ctypes.c_int32), ("hmax2", ctypes.c_int32),
                ("S", ctypes.c_float * 6)]


def ewald_params(L: float, M: float, com, G: float = 1.0, alpha: float = 0.0, nrep: int = 1,
                 hmax2: int = 10, S=None) -> EwaldParams:
    p = EwaldParams()
    p.L, p.G, p.M, p.alpha, p.nrep, p.hmax2 = float(L), float(G), float(M), float(alpha), int(nrep), int(hmax2)
    for d in range(3):
        p.com[d] = float(com[d])
    if S is not None:
        for k in range(6):
            p.S[k] = float(S[k])
    return p


class GcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gcharm status {status}: {msg}")
        self.status = status


class ForceParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("G", ctypes.c_float), ("soft_eps", ctypes.c_float),
                ("n_types", ctypes.c_int32), ("eps_t", ctypes.c_void_p), ("sig_t", ctypes.c_void_p),
                ("mass_t", ctypes.c_void_p), ("r_cut", ctypes.c_float), ("schedule", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("targets_per_lane", ctypes.c_int32), ("n_nodes", ctypes.c_int32), ("want_potential", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("aggregation", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
VP, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
PI32 = ctypes.POINTER(ctypes.c_int32)
PI64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    """The loaded libgcharm.so (raises GcError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GcError(GC_E_STATE, f"{LIB_PATH} is missing: run __graft_entry__.build() (no fallback exists)")
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7).  Loading torch first
    # makes libgcharm.so bind to that runtime, so torch's device pointers and stream handles are
    # valid in the library and the process holds a single HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "gc_version": (ctypes.c_char_p, []),
        "gc_init": (I32, [ctypes.c_int, VP, VP, VP, ctypes.POINTER(VP)]),
        "gc_debug_inject_error": (I32, [VP, ctypes.c_int]),
        "gc_debug_step_waits": (I32, [VP, ctypes.c_uint32, I32]),
        "gc_batch_status": (I32, [VP, VP]),
        "gc_graph_status": (I32, [VP, VP]),
        "gc_finalize": (I32, [VP]),
        "gc_last_error": (ctypes.c_char_p, [VP]),
        "gc_pool_create": (I32, [VP, I32, I32, ctypes.POINTER(VP)]),
        "gc_pool_destroy": (I32, [VP]),
        "gc_pool_set_source": (I32, [VP, VP]),
        "gc_pool_set_host_source": (I32, [VP, VP]),
        "gc_pool_query_mirror": (I32, [VP, VP, VP]),
        "gc_pool_place": (I32, [VP, VP, VP, I32, VP]),
        "gc_pool_reset": (I32, [VP, VP]),
        "gc_pool_evict": (I32, [VP, VP, I32, VP]),
        "gc_pool_evict_staged": (I32, [VP, VP, VP]),
        "gc_pool_query": (I32, [VP, VP, VP]),
        "gc_pool_device_ptrs": (I32, [VP, ctypes.POINTER(VP), ctypes.POINTER(VP)]),
        "gc_batch_create": (I32, [VP, I32, I32, ctypes.POINTER(VP)]),
        "gc_batch_destroy": (I32, [VP]),
        "gc_batch_reset": (I32, [VP]),
        "gc_submit_tasks": (I32, [VP, VP, I32, VP, I32, VP, I32]),
        "gc_submit_tasks_device": (I32, [VP, VP, I32, VP, I32, VP, I32, I32, VP]),
        "gc_walk_tasks": (I32, [VP, I32, I32, I32, VP, I32, VP, VP, VP, VP, VP]),
        "gc_batch_commit": (I32, [VP, VP]),
        "gc_batch_sizes": (I32, [VP, PI64]),
        "gc_reorganize": (I32, [VP, VP, I32, I32, VP, VP]),
        "gc_batch_maps": (I32, [VP, PI64, VP, VP, VP, VP, VP, VP, VP, VP, VP]),
        "gc_launch_combined": (I32, [VP, ctypes.POINTER(ForceParams), VP, VP, VP]),
        "gc_zero_f32": (I32, [VP, VP, I64, VP]),
        "gc_backward": (I32, [VP, ctypes.POINTER(ForceParams), VP, VP, I32, VP, VP, VP, VP, VP]),
        "gc_graph_capture": (I32, [VP, I32, ctypes.POINTER(VP), ctypes.POINTER(VP), VP, ctypes.POINTER(ForceParams),
                                   VP, VP, I32, ctypes.POINTER(VP), ctypes.POINTER(VP), VP, VP, ctypes.POINTER(VP)]),
        "gc_graph_launch": (I32, [VP, VP]),
        "gc_graph_destroy": (I32, [VP]),
        "gc_autotune": (I32, [VP, ctypes.POINTER(ForceParams), VP, VP, I32, VP, ctypes.POINTER(ForceParams),
                              ctypes.c_char_p, PI32, VP]),
        "gc_occupancy": (I32, [VP, ctypes.POINTER(ForceParams), PI32, PI32]),
        "gc_lj_count_pairs": (I32, [VP, ctypes.c_float, PI64, VP]),
        "gc_launch_ewald": (I32, [VP, ctypes.POINTER(EwaldParams), VP, VP]),
        "gc_hybrid_create": (I32, [ctypes.POINTER(VP)]),
        "gc_hybrid_destroy": (I32, [VP]),
        "gc_hybrid_record": (I32, [VP, I32, I64, ctypes.c_double]),
        "gc_hybrid_split": (I32, [VP, VP, I32, PI32, PI64]),
        "gc_hybrid_state": (I32, [VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), PI64, PI64]),
        "gc_lj_forces_cpu": (I32, [VP, I32, VP, I32, VP, I32, I32, VP, VP, VP, ctypes.c_float, VP, I32]),
        "gc_combiner_create": (I32, [I32, ctypes.POINTER(VP)]),
        "gc_combiner_destroy": (I32, [VP]),
        "gc_combiner_arrive": (I32, [VP, ctypes.c_double, I64]),
        "gc_combiner_poll": (I32, [VP, ctypes.c_double, PI64, PI32]),
        "gc_combiner_state": (I32, [VP, PI64, ctypes.POINTER(ctypes.c_double), PI64, PI64]),
        "gc_tree_walk": (I32, [VP, I32, VP, VP, VP, VP, I32, I32, VP, ctypes.c_double, VP, VP, VP, I64, VP, I64,
                               PI64, VP]),
        "gc_tree_walk_noalloc": (I32, [VP, I32, VP, VP, VP, VP, I32, I32, VP, ctypes.c_double, VP, VP, VP, I64, VP,
                                       I64, PI64, VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(x) -> int | None:
    """Device/host address of a torch tensor, numpy array or int (None passes NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s) -> int | None:
    if s is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:  # noqa: BLE001 - no torch GPU: default stream
            return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def torch_allocator(device: int = 0):
    """(alloc, free) hooks over torch's caching allocator (memory on the current stream of `device`)."""
    import torch

    def alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:  # noqa: BLE001 - out of memory: the library reports GC_E_NOMEM
            return None

    def free(ptr, _user):
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


class Context:
    """One device context (gc_init / gc_finalize).

    allocator: None (the library's hipMalloc / hipFree), "torch" (torch's caching allocator), or a pair
    of Python callables (alloc(nbytes, user) -> int address or None, free(address, user)).
    """

    def __init__(self, device: int = 0, allocator=None):
        self.h = VP()
        self._hooks = None
        a = f = None
        if allocator is not None:
            pa, pf = torch_allocator(device) if allocator == "torch" else allocator
            self._hooks = (ALLOC_FN(pa), FREE_FN(pf))  # kept alive as long as the context
            a, f = ctypes.cast(self._hooks[0], VP), ctypes.cast(self._hooks[1], VP)
        st = lib().gc_init(device, a, f, None, ctypes.byref(self.h))
        if st != GC_OK:
            raise GcError(st, f"gc_init({device}) failed")

    def inject_error(self, hip_error: int = 1):
        """Test hook: the next call reports an asynchronous device error (gc_debug_inject_error)."""
        st = lib().gc_debug_inject_error(self.h, int(hip_error))
        if st != GC_OK:
            raise GcError(st, "gc_debug_inject_error")

    def step_waits(self, fail_spins: int = 0, fail_round: int = -1):
        """Test hook for later whole-step captures (gc_debug_step_waits); fail_round -1 turns it off."""
        self.check(lib().gc_debug_step_waits(self.h, int(fail_spins), int(fail_round)), "gc_debug_step_waits")

    def check(self, st: int, what: str = ""):
        if st != GC_OK:
            raise GcError(st, f"{what}: {lib().gc_last_error(self.h).decode()}")

    def zero(self, t, stream=None):
        self.check(lib().gc_zero_f32(self.h, _ptr(t), t.numel(), _stream(stream)), "gc_zero_f32")

    def occupancy(self, prm: ForceParams):
        b, n = ctypes.c_int32(), ctypes.c_int32()
        self.check(lib().gc_occupancy(self.h, ctypes.byref(prm), ctypes.byref(b), ctypes.byref(n)), "gc_occupancy")
        return b.value, n.value

    def close(self):
        if self.h:
            lib().gc_finalize(self.h)
            self.h = VP()


class Combiner:
    """The arrival-rate combining policy (gc_combiner_*): host logic, the caller's clock in seconds."""

    def __init__(self, max_size: int):
        self.h = VP()
        st = lib().gc_combiner_create(int(max_size), ctypes.byref(self.h))
        if st != GC_OK:
            raise GcError(st, f"gc_combiner_create({max_size})")

    def arrive(self, t: float, n: int = 1):
        st = lib().gc_combiner_arrive(self.h, float(t), int(n))
        if st != GC_OK:
            raise GcError(st, f"gc_combiner_arrive(t={t}, n={n})")

    def poll(self, t: float) -> tuple[int, int]:
        """(requests to combine now, reason: 0 none, 1 max_size reached, 2 idle)."""
        k, why = ctypes.c_int64(), ctypes.c_int32()
        st = lib().gc_combiner_poll(self.h, float(t), ctypes.byref(k), ctypes.byref(why))
        if st != GC_OK:
            raise GcError(st, f"gc_combiner_poll(t={t})")
        return k.value, why.value

    def state(self) -> dict:
        w, mi, nf, ni = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        st = lib().gc_combiner_state(self.h, ctypes.byref(w), ctypes.byref(mi), ctypes.byref(nf), ctypes.byref(ni))
        if st != GC_OK:
            raise GcError(st, "gc_combiner_state")
        return {"waiting": w.value, "max_interval": mi.value, "n_full": nf.value, "n_idle": ni.value}

    def destroy(self):
        if self.h:
            lib().gc_combiner_destroy(self.h)
            self.h = VP()


DEVICE_CPU, DEVICE_GPU = 0, 1


class Hybrid:
    """Dynamic CPU/GPU scheduling of work requests by running per-item times (gc_hybrid_*)."""

    def __init__(self):
        self.h = VP()
        st = lib().gc_hybrid_create(ctypes.byref(self.h))
        if st != GC_OK:
            raise GcError(st, "gc_hybrid_create")

    def record(self, device: int, items: int, seconds: float):
        st = lib().gc_hybrid_record(self.h, int(device), int(items), float(seconds))
        if st != GC_OK:
            raise GcError(st, f"gc_hybrid_record(device={device}, items={items}, seconds={seconds})")

    def split(self, items) -> tuple[int, int]:
        """(requests at the front of the queue that go to the CPU, their items)."""
        it = np.ascontiguousarray(items, dtype=np.int64)
        k, ic = ctypes.c_int32(), ctypes.c_int64()
        st = lib().gc_hybrid_split(self.h, it.ctypes.data if it.size else None, int(it.size), ctypes.byref(k),
                                   ctypes.byref(ic))
        if st != GC_OK:
            raise GcError(st, "gc_hybrid_split")
        return k.value, ic.value

    def state(self) -> dict:
        tc, tg, rc, rg = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        st = lib().gc_hybrid_state(self.h, ctypes.byref(tc), ctypes.byref(tg), ctypes.byref(rc), ctypes.byref(rg))
        if st != GC_OK:
            raise GcError(st, "gc_hybrid_state")
        return {"tau_cpu": tc.value, "tau_gpu": tg.value, "runs_cpu": rc.value, "runs_gpu": rg.value}

    def destroy(self):
        if self.h:
            lib().gc_hybrid_destroy(self.h)
            self.h = VP()


def lj_forces_cpu(tasks: np.ndarray, ranges: np.ndarray, rec: np.ndarray, eps_t, sig_t, mass_t, r_cut: float,
                  acc: np.ndarray, n_threads: int = 0):
    """acc (host float32 [n_ids, 4]) += accelerations of the given LJ tasks on the CPU (gc_lj_forces_cpu)."""
    tasks = np.ascontiguousarray(tasks, dtype=TASK_DTYPE)
    ranges = np.ascontiguousarray(ranges, dtype=np.int32).reshape(-1, 2)
    rec = np.ascontiguousarray(rec, dtype=np.float32)
    e, sgm, m = (np.ascontiguousarray(x, dtype=np.float32) for x in (eps_t, sig_t, mass_t))
    assert acc.dtype == np.float32 and acc.flags.c_contiguous and acc.shape == (rec.shape[0], 4)
    st = lib().gc_lj_forces_cpu(tasks.ctypes.data, int(tasks.size), ranges.ctypes.data, int(ranges.shape[0]),
                                rec.ctypes.data, int(rec.shape[0]), int(e.size), e.ctypes.data, sgm.ctypes.data,
                                m.ctypes.data, float(r_cut), acc.ctypes.data, int(n_threads))
    if st != GC_OK:
        raise GcError(st, "gc_lj_forces_cpu")


def tree_walk(ctx: "Context", node_range, node_com, node_side, rec, bucket_node, theta: float, stream=None,
              noalloc: bool = False):
    """Barnes-Hut lists of every bucket on the device (gc_tree_walk, or gc_tree_walk_noalloc); device
    tensors in, device tensors out: (n_first int32 [nb + 1], node_idx int32, r_first int32 [nb + 1],
    ranges int32 [., 2])."""
    import torch
    fn = lib().gc_tree_walk_noalloc if noalloc else lib().gc_tree_walk
    name = "gc_tree_walk_noalloc" if noalloc else "gc_tree_walk"
    dev = node_range.device
    nb = int(bucket_node.numel())
    n_first = torch.empty(nb + 1, dtype=torch.int32, device=dev)
    r_first = torch.empty(nb + 1, dtype=torch.int32, device=dev)
    totals = (ctypes.c_int64 * 2)()
    args = (ctx.h, int(node_range.shape[0]), _ptr(node_range), _ptr(node_com), _ptr(node_side), _ptr(rec),
            int(rec.shape[0]), nb, _ptr(bucket_node), float(theta), _ptr(n_first), _ptr(r_first))
    st = fn(*args, None, 0, None, 0, totals, _stream(stream))
    if st == GC_E_FULL:  # sized by the first call's counts
        node_idx = torch.empty(max(totals[0], 1), dtype=torch.int32, device=dev)
        ranges = torch.empty((max(totals[1], 1), 2), dtype=torch.int32, device=dev)
        st = fn(*args, _ptr(node_idx), int(totals[0]), _ptr(ranges), int(totals[1]), totals, _stream(stream))
    else:
        node_idx = torch.empty(1, dtype=torch.int32, device=dev)
        ranges = torch.empty((1, 2), dtype=torch.int32, device=dev)
    ctx.check(st, name)
    return n_first, node_idx[:totals[0]], r_first, ranges[:totals[1]]


def walk_tasks(ctx: "Context", b0: int, b1: int, bucket_node, node_range, n_first, r_first, stream=None):
    """gc_task records of buckets [b0, b1) of a list walk, as a device uint8 tensor (gc_walk_tasks)."""
    import torch
    out = torch.empty(max(b1 - b0, 1) * TASK_DTYPE.itemsize, dtype=torch.uint8, device=bucket_node.device)
    ctx.check(lib().gc_walk_tasks(ctx.h, int(bucket_node.numel()), int(b0), int(b1), _ptr(bucket_node),
                                  int(node_range.shape[0]),
                                  _ptr(node_range), _ptr(n_first), _ptr(r_first), _ptr(out), _stream(stream)),
              "gc_walk_tasks")
    return out[:(b1 - b0) * TASK_DTYPE.itemsize]


class Pool:
    """Device record pool + chare table (gc_pool_*)."""

    def __init__(self, ctx: Context, n_ids: int, capacity: int):
        self.ctx = ctx
        self.n_ids, self.capacity = n_ids, capacity
        self.h = VP()
        ctx.check(lib().gc_pool_create(ctx.h, n_ids, capacity, ctypes.byref(self.h)), "gc_pool_create")
        self._src = None

    def set_source(self, records):
        self._src = records  # keep alive
        self.ctx.check(lib().gc_pool_set_source(self.h, _ptr(records)), "gc_pool_set_source")

    def set_host_source(self, records: np.ndarray):
        """Host records (float32 [n_ids, 4], any host memory) staged by host-issued copies of the missing
        records only (gc_pool_set_host_source)."""
        assert records.dtype == np.float32 and records.flags.c_contiguous and records.shape == (self.n_ids, 4)
        self._src = records  # keep alive
        self.ctx.check(lib().gc_pool_set_host_source(self.h, records.ctypes.data), "gc_pool_set_host_source")

    def query_mirror(self, stream=None) -> np.ndarray:
        """The host mirror of the chare table of a host-source pool (gc_pool_query_mirror)."""
        out = np.empty(self.n_ids, np.int32)
        self.ctx.check(lib().gc_pool_query_mirror(self.h, out.ctypes.data, _stream(stream)), "gc_pool_query_mirror")
        return out

    def place(self, ids_dev, slots_dev, stream=None):
        self.ctx.check(lib().gc_pool_place(self.h, _ptr(ids_dev), _ptr(slots_dev), int(ids_dev.numel()),
                                           _stream(stream)), "gc_pool_place")

    def reset(self, stream=None):
        self.ctx.check(lib().gc_pool_reset(self.h, _stream(stream)), "gc_pool_reset")

    def evict(self, ids_dev, stream=None):
        self.ctx.check(lib().gc_pool_evict(self.h, _ptr(ids_dev), int(ids_dev.numel()), _stream(stream)),
                       "gc_pool_evict")

    def evict_staged(self, batch, stream=None):
        self.ctx.check(lib().gc_pool_evict_staged(self.h, batch.h, _stream(stream)), "gc_pool_evict_staged")

    def query(self, stream=None) -> np.ndarray:
        out = np.empty(self.n_ids, np.int32)
        self.ctx.check(lib().gc_pool_query(self.h, out.ctypes.data, _stream(stream)), "gc_pool_query")
        return out

    def device_ptrs(self):
        r, s = VP(), VP()
        self.ctx.check(lib().gc_pool_device_ptrs(self.h, ctypes.byref(r), ctypes.byref(s)), "gc_pool_device_ptrs")
        return r.value, s.value

    def destroy(self):
        if self.h:
            lib().gc_pool_destroy(self.h)
            self.h = VP()


def tasks_from_csr(i_begin, i_count, j_first, j_nr, n_first=None, n_count=None, flags=None, shift=None) -> np.ndarray:
    """Pack per-task CSR columns into gc_task records."""
    T = len(i_begin)
    t = np.zeros(T, TASK_DTYPE)
    t["i_begin"], t["i_count"], t["j_first"], t["j_nranges"] = i_begin, i_count, j_first, j_nr
    if n_first is not None:
        t["n_first"], t["n_count"] = n_first, n_count
    if flags is not None:
        t["flags"] = flags
    if shift is not None:
        t["shift"] = shift
    return t


class Batch:
    """A combined work request (gc_batch_*, gc_submit_tasks, gc_reorganize, gc_launch_combined, gc_backward)."""

    def __init__(self, ctx: Context, kind: int, n_ids: int):
        self.ctx = ctx
        self.kind, self.n_ids = kind, n_ids
        self.h = VP()
        ctx.check(lib().gc_batch_create(ctx.h, kind, n_ids, ctypes.byref(self.h)), "gc_batch_create")

    def submit(self, tasks: np.ndarray, ranges: np.ndarray, node_idx: np.ndarray | None = None):
        tasks = np.ascontiguousarray(tasks, TASK_DTYPE)
        ranges = np.ascontiguousarray(ranges, np.int32).reshape(-1, 2)
        node_idx = np.ascontiguousarray(np.zeros(0, np.int32) if node_idx is None else node_idx, np.int32)
        self.ctx.check(lib().gc_submit_tasks(self.h, tasks.ctypes.data, len(tasks), ranges.ctypes.data,
                                             ranges.shape[0], node_idx.ctypes.data, node_idx.size), "gc_submit_tasks")

    def reset(self):
        """Drop every submitted task (gc_batch_reset)."""
        self.ctx.check(lib().gc_batch_reset(self.h), "gc_batch_reset")

    def submit_device(self, tasks_dev, ranges_dev, node_idx_dev, n_nodes: int, stream=None):
        """Device tensors: tasks (uint8 / int32 view of gc_task records, n_tasks * 40 bytes), ranges int32
        [n, 2], node_idx int32 (gc_submit_tasks_device)."""
        n_tasks = (tasks_dev.numel() * tasks_dev.element_size()) // TASK_DTYPE.itemsize
        self.ctx.check(lib().gc_submit_tasks_device(self.h, _ptr(tasks_dev), int(n_tasks), _ptr(ranges_dev),
                                                    int(ranges_dev.numel() // 2), _ptr(node_idx_dev),
                                                    int(node_idx_dev.numel()), int(n_nodes), _stream(stream)),
                       "gc_submit_tasks_device")

    def commit(self, stream=None):
        self.ctx.check(lib().gc_batch_commit(self.h, _stream(stream)), "gc_batch_commit")

    def sizes(self) -> dict:
        out = np.zeros(5, np.int64)
        self.ctx.check(lib().gc_batch_sizes(self.h, out.ctypes.data_as(PI64)), "gc_batch_sizes")
        return dict(tasks=int(out[0]), ranges=int(out[1]), node_refs=int(out[2]), direct=int(out[3]),
                    targets=int(out[4]))

    def reorganize(self, pool: Pool, mode: int, check_capacity: bool = True, stream=None, side=None):
        """side: stream of the staging copies of a host-source pool (None: `stream`)."""
        self.ctx.check(lib().gc_reorganize(self.h, pool.h, mode, 1 if check_capacity else 0, _stream(stream),
                                           None if side is None else _stream(side)), "gc_reorganize")

    def maps(self, stream=None) -> dict:
        sz = self.sizes()
        counts = np.zeros(2, np.int64)
        n = self.n_ids
        U = np.empty(max(n, 1), np.int32)
        pos = np.empty(max(n, 1), np.int32)
        missing = np.empty(max(n, 1), np.int32)
        new_slot = np.empty(max(n, 1), np.int32)
        pr = np.empty((max(sz["ranges"], 1), 2), np.int32)
        pib = np.empty(max(sz["tasks"], 1), np.int32)
        il = np.empty(max(sz["targets"], 1), np.int32)
        jl = np.empty(max(sz["direct"], 1), np.int32)
        self.ctx.check(lib().gc_batch_maps(self.h, counts.ctypes.data_as(PI64), U.ctypes.data, pos.ctypes.data,
                                           missing.ctypes.data, new_slot.ctypes.data, pr.ctypes.data, pib.ctypes.data,
                                           il.ctypes.data, jl.ctypes.data, _stream(stream)), "gc_batch_maps")
        nu, nm = int(counts[0]), int(counts[1])
        return dict(U=U[:nu], pos=pos[:n], missing=missing[:nm], new_slot=new_slot[:nm], pranges=pr[:sz["ranges"]],
                    pi_begin=pib[:sz["tasks"]], ilist=il[:sz["targets"]], jlist=jl[:sz["direct"]])

    def launch(self, prm: ForceParams, nodes, acc, stream=None):
        p = with_nodes(prm, nodes)
        self.ctx.check(lib().gc_launch_combined(self.h, ctypes.byref(p), _ptr(nodes), _ptr(acc), _stream(stream)),
                       "gc_launch_combined")

    def lj_count_pairs(self, r_cut: float, stream=None) -> int:
        """In-cutoff pairs of this Lennard-Jones batch (gc_lj_count_pairs)."""
        n = ctypes.c_int64()
        self.ctx.check(lib().gc_lj_count_pairs(self.h, float(r_cut), ctypes.byref(n), _stream(stream)),
                       "gc_lj_count_pairs")
        return n.value

    def status(self, stream=None):
        """Raises GcError if a device-side wait gave up or a backward met bad node ranges (gc_batch_status)."""
        self.ctx.check(lib().gc_batch_status(self.h, _stream(stream)), "gc_batch_status")

    def ewald(self, prm: "EwaldParams", acc, stream=None):
        """acc += the Ewald correction at every target of the batch (gc_launch_ewald)."""
        self.ctx.check(lib().gc_launch_ewald(self.h, ctypes.byref(prm), _ptr(acc), _stream(stream)), "gc_launch_ewald")

    def backward(self, prm: ForceParams, nodes, node_range, n_nodes: int, cot, gpos, gmass, gparam=None,
                 stream=None):
        prm = with_nodes(prm, nodes)
        self.ctx.check(lib().gc_backward(self.h, ctypes.byref(prm), _ptr(nodes), _ptr(node_range), int(n_nodes),
                                         _ptr(cot), _ptr(gpos), _ptr(gmass), _ptr(gparam), _stream(stream)),
                       "gc_backward")

    def autotune(self, base: ForceParams, nodes, acc, reps: int = 3, stream=None, cache_path: str | None = None):
        """(best parameters, times of the 36 shapes and 4 aggregation counts in ms (NaN: not timed), whether the
        result came from the tuning cache) (gc_autotune)."""
        times = np.full(40, np.nan, np.float32)
        best = ForceParams()
        hit = ctypes.c_int32(0)
        base = with_nodes(base, nodes)
        self.ctx.check(lib().gc_autotune(self.h, ctypes.byref(base), _ptr(nodes), _ptr(acc), reps, times.ctypes.data,
                                         ctypes.byref(best), None if cache_path is None else cache_path.encode(),
                                         ctypes.byref(hit), _stream(stream)), "gc_autotune")
        return best, times, bool(hit.value)

    def destroy(self):
        if self.h:
            lib().gc_batch_destroy(self.h)
            self.h = VP()


class Graph:
    """A captured sequence of (reorganise, combined pass) steps (gc_graph_*)."""

    def __init__(self, ctx: Context, batches, pools, modes, prm: ForceParams, nodes, acc, pre_reset: bool = False,
                 places=None, stream=None, fixture: int | None = None):
        """fixture: FIXTURE_* (default: RESET_PLACE when pre_reset, else NONE)."""
        n = len(batches)
        self.ctx = ctx
        self.h = VP()
        B = (VP * n)(*[b.h.value for b in batches])
        P = (VP * n)(*[p.h.value for p in pools])
        M = np.ascontiguousarray(modes, np.int32)
        if fixture is None:
            fixture = FIXTURE_RESET_PLACE if pre_reset else FIXTURE_NONE
        if places is not None:
            self._keep = places
            ids = (VP * n)(*[_ptr(pl[0]) for pl in places])
            sl = (VP * n)(*[_ptr(pl[1]) for pl in places])
            pn = np.array([int(pl[0].numel()) for pl in places], np.int32)
            pn_ptr = pn.ctypes.data
            self._pn = pn
        else:
            ids = sl = None
            pn_ptr = None
        prm = with_nodes(prm, nodes)
        self.ctx.check(lib().gc_graph_capture(ctx.h, n, B, P, M.ctypes.data, ctypes.byref(prm), _ptr(nodes), _ptr(acc),
                                              fixture, ids, sl, pn_ptr, _stream(stream),
                                              ctypes.byref(self.h)), "gc_graph_capture")

    def launch(self, stream=None):
        self.ctx.check(lib().gc_graph_launch(self.h, _stream(stream)), "gc_graph_launch")

    def status(self, stream=None):
        """Raises GcError if a bounded wait gave up in a launch since capture (gc_graph_status)."""
        self.ctx.check(lib().gc_graph_status(self.h, _stream(stream)), "gc_graph_status")

    def destroy(self):
        if self.h:
            lib().gc_graph_destroy(self.h)
            self.h = VP()


def with_nodes(prm: ForceParams, nodes) -> ForceParams:
    """A copy of prm whose n_nodes is the node table's record count (12 floats per node)."""
    p = ForceParams.from_buffer_copy(prm)
    if nodes is not None and prm.kind in (FORCE_GRAV_MONO, FORCE_GRAV_QUAD):
        p.n_nodes = int(nodes.numel() if hasattr(nodes, "numel") else np.asarray(nodes).size) // 12
    return p


def grav_params(order: int = 2, G: float = 1.0, eps: float = 0.01, schedule: int = 0, tile: int = 0,
                waves_per_block: int = 0, grid_blocks: int = 0, targets_per_lane: int = 0, want_potential: int = 0,
                deterministic: int = 0, aggregation: int = 0) -> ForceParams:
    """Gravity parameters; n_nodes is filled in from the node table by the calls that take one."""
    p = ForceParams()
    p.kind = FORCE_GRAV_QUAD if order == 2 else FORCE_GRAV_MONO
    p.G, p.soft_eps = G, eps
    p.schedule, p.tile, p.waves_per_block, p.grid_blocks = schedule, tile, waves_per_block, grid_blocks
    p.targets_per_lane = targets_per_lane
    p.want_potential, p.deterministic = want_potential, deterministic
    p.aggregation = aggregation
    return p


def lj_params(eps_t, sig_t, mass_t, r_cut: float, schedule: int = 0, grid_blocks: int = 0, want_potential: int = 0,
              deterministic: int = 0) -> ForceParams:
    """eps_t, sig_t, mass_t: device float32 tensors (kept alive by the caller)."""
    p = ForceParams()
    p.kind = FORCE_LJ
    p.n_types = int(eps_t.numel())
    p.eps_t, p.sig_t, p.mass_t = _ptr(eps_t), _ptr(sig_t), _ptr(mass_t)
    p.r_cut = r_cut
    p.schedule, p.grid_blocks = schedule, grid_blocks
    p.want_potential, p.deterministic = want_potential, deterministic
    return p
