// Host runtime behind the C ABI in gcharm.h: contexts, the device pool and its
// chare table, batches (combined work requests), the reorganisation pipeline,
// the combined launches, HIP graph capture and the autotuner.
#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "gc_internal.h"
#include "walk.h"

using namespace gc;

namespace {
// The caller's device allocator (gc_init); both NULL: hipMalloc / hipFree.
struct AllocHooks {
  gc_alloc_fn alloc = nullptr;
  gc_free_fn free = nullptr;
  void* user = nullptr;
};

// Device buffer that only grows, allocated through its context's hooks.  Memory goes back to the
// caller's allocator only after the device is idle, since a caching allocator may hand it out again
// at once to work on another stream.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const AllocHooks* h = nullptr;
  hipError_t give_back() {
    hipError_t e = hipSuccess;
    if (p) {
      if (h && h->alloc) {
        e = hipDeviceSynchronize();
        h->free(p, h->user);
      } else {
        e = hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
    return e;
  }
  hipError_t ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    hipError_t e = give_back();
    if (e != hipSuccess) return e;
    size_t b = want < 256 ? 256 : want;
    if (h && h->alloc) {
      p = h->alloc(b, h->user);
      if (!p) return hipErrorOutOfMemory;
    } else {
      e = hipMalloc(&p, b);
      if (e != hipSuccess) {
        p = nullptr;
        return e;
      }
    }
    bytes = b;
    return hipSuccess;
  }
  void release() { (void)give_back(); }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Pinned host buffer (hipHostMalloc) that only grows: the staging area of host-issued copies.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    release();
    size_t b = want < 4096 ? 4096 : want + want / 4;
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// An event created on first use (timing off), destroyed with its owner.
struct Event {
  hipEvent_t e = nullptr;
  bool recorded = false;
  hipError_t record(hipStream_t s) {
    if (!e) {
      hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (r != hipSuccess) {
        e = nullptr;
        return r;
      }
    }
    recorded = true;
    return hipEventRecord(e, s);
  }
  hipError_t wait(hipStream_t s) const { return recorded ? hipStreamWaitEvent(s, e, 0) : hipSuccess; }
  hipError_t sync() const { return recorded ? hipEventSynchronize(e) : hipSuccess; }
  void destroy() {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
    recorded = false;
  }
};

}  // namespace

struct gc_ctx_ {
  int device = 0;
  int n_cu = 0;
  bool poisoned = false;
  hipError_t injected = hipSuccess;  // test hook: an error that the next call reports as asynchronous
  std::string err;
  AllocHooks hooks;
  DevBuf walk_keep;  // the list walk's per-bucket room, kept between calls
  void* walk_scratch = nullptr;  // device address of this device's fixed walk scratch (no-allocation walk)
  // test hook for the whole-step schedule, taken by the next capture: a round whose force items wait
  // for a count that is never reached (-1: none), and the bound on those waits (0: the default)
  int32_t step_fail_round = -1;
  uint32_t step_fail_spins = 0;
};

namespace {

gc_status set_err(gc_ctx c, gc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

gc_status hip_fail(gc_ctx c, hipError_t e, const char* what) {
  if (c) c->poisoned = true;
  return set_err(c, GC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define GC_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

#define GC_ENTER(ctx)                                                                   \
  do {                                                                                  \
    if (!(ctx)) return GC_E_INVAL;                                                      \
    if ((ctx)->poisoned) return set_err((ctx), GC_E_STATE, "context poisoned by an earlier device error"); \
    (ctx)->err.clear();                                                                 \
    if ((ctx)->injected != hipSuccess) {                                                \
      const hipError_t inj_ = (ctx)->injected;                                          \
      (ctx)->injected = hipSuccess;                                                     \
      return hip_fail((ctx), inj_, "asynchronous device error (injected)");             \
    }                                                                                   \
  } while (0)

inline int64_t pad_to(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

struct gc_pool_ {
  gc_ctx ctx = nullptr;
  int32_t n_ids = 0, cap = 0;
  DevBuf rec, slot_of, occ;
  const float4* src = nullptr;
  bool src_device = false;
  // host source (gc_pool_set_host_source): records staged by host-issued copies, and the host's
  // mirror of the chare table that tells it which records are missing without asking the device
  const float4* host_src = nullptr;
  std::vector<int32_t> m_slot_of;  // by id, -1: not resident
  std::vector<uint64_t> m_free;    // bit s of word s / 64: slot s free
  int64_t m_nfree = 0;
  size_t m_lo = 0;                 // no free slot below word m_lo
  bool mirror_ok = false;          // false: the device changed the table without the host tracking it
  PinnedBuf pin;                   // gc_pool_place staging
  DevBuf tmp;
  Event ev_pin;
  std::vector<DevBuf*> bufs() { return {&rec, &slot_of, &occ, &tmp}; }
};

struct gc_batch_ {
  gc_ctx ctx = nullptr;
  // host-side: the batch's last reorganisation may have left staged records in its pool (cleared by
  // gc_pool_evict_staged and by a whole-step or rounds launch under the evicting fixture, which
  // stages nothing that outlives its round)
  bool staged_live = false;
  int32_t kind = GC_KIND_GRAV;
  int32_t n_ids = 0;
  std::vector<gc_task> tasks;
  std::vector<int32_t> ranges;   // pairs
  std::vector<int32_t> nodes;
  int64_t n_direct = 0, n_targets = 0;
  int32_t nt = 0, nr = 0, nn = 0;  // tasks, ranges and node refs submitted (host or device)
  bool committed = false;
  // device submission (gc_submit_tasks_device): tasks and lists arrive in d_tasks / d_ranges / d_nodes
  // and the commit runs on the device; the host vectors (tasks, ranges, nodes, hU, h_order, h_pibeg)
  // are filled from the device only when a host-side step needs them (host_lists)
  bool dev_sub = false, host_lists = true;
  int32_t dev_n_nodes = 0;
  DevBuf dc_dc, dc_cost, dc_diff, dc_bs, dc_ns, dc_tot, d_pos;
  // fixed at commit: the sorted union U and the packed-space ranges and first targets
  std::vector<int32_t> hU;
  std::vector<int32_t> h_order, h_pibeg;  // launch order of the tasks and their first packed targets
  int32_t u = 0, max_direct = 0;
  DevBuf d_tasks, d_ranges, d_nodes, d_ioff, d_joff, d_order, d_runs, d_U, pranges, pibeg;
  int32_t n_runs = 0;
  // Lennard-Jones gather form (possible when any two target ranges are equal or disjoint): the
  // target ranges and, per range, its tasks and sides; cover: the ranges hold every id
  DevBuf d_ljtgt, d_ljent;
  int32_t n_ljtgt = 0;
  bool lj_gather = false, lj_cover = false;
  bool ranks_ready = false;      // union ranks of the address-list entries (built on first use)
  DevBuf d_irank, d_jrank;
  // reorganisation buffers
  DevBuf uslot, missing, mslot, free_list, state, packed, ilist, jlist, queue;
  DevBuf force, ppart;  // adjoint scratch: recomputed LJ forces, LJ parameter partials
  // gravity adjoint: per-visit gradient records, the node visits grouped by node and cut into chunks,
  // the chunk sums, and the direct visits grouped by source id (built on the first backward call)
  DevBuf vnode, vdir, nvis, nchunks, nchunk_first, npart, dvis, dkey;
  int32_t adj_nodes = -1, adj_chunks = 0;  // node count the indices were built for (-1: none)
  DevBuf stat;  // device-side error words: [0] node ranges the adjoint found out of bounds
  int32_t max_node = -1;  // largest node index submitted
  // state of the last reorganisation
  int32_t mode = -1;
  gc_pool pool = nullptr;
  const float4* rec = nullptr;
  // host-staged reorganisation: the missing records packed on the host (pin), their device copy
  // (staged), the copy's completion (ev_copy) and the last compute-stream work that read this
  // batch's staged or packed records (ev_use, which the next copy waits for)
  PinnedBuf pin;
  DevBuf staged;
  Event ev_copy, ev_use;
  bool host_staged = false;
  std::vector<int32_t> h_missing, h_mslot;  // the last host-staged call's missing ids and their slots
  std::vector<DevBuf*> bufs() {
    return {&d_tasks, &d_ranges, &d_nodes, &d_ioff, &d_joff, &d_order, &d_runs, &d_U, &pranges, &pibeg, &d_irank,
            &d_jrank, &uslot, &missing, &mslot, &free_list, &state, &packed, &ilist, &jlist, &queue, &force, &ppart,
            &vnode, &vdir, &nvis, &nchunks, &nchunk_first, &npart, &dvis, &dkey, &d_ljtgt, &d_ljent, &stat, &staged,
            &dc_dc, &dc_cost, &dc_diff, &dc_bs, &dc_ns, &dc_tot, &d_pos};
  }
};

struct gc_graph_ {
  gc_ctx ctx = nullptr;
  std::vector<gc_pool> pools;      // pools the graph changes (their host mirrors go stale at each launch)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // whole-step / rounds schedule under the evicting fixture: the same graph without the kernel that
  // evicts what the last batch left staged, launched when the host knows nothing is staged
  hipGraph_t graph_noevict = nullptr;
  hipGraphExec_t exec_noevict = nullptr;
  std::vector<gc_batch> batches;  // the captured batches (staging bookkeeping)
  int32_t fixture = GC_FIXTURE_NONE;
  bool step_form = false;
  DevBuf step_items, step_rounds, step_ctr, step_fl;  // whole-step persistent schedule
  DevBuf round_items, round_args;  // rounds schedule: the combined pass's items and per-round arguments
  std::vector<hipStream_t> side;   // capture-time side streams (combined passes of successive steps overlap)
  std::vector<hipEvent_t> events;
  std::vector<const int32_t*> err_words;  // the error words of the batches the graph reorganises
  std::vector<DevBuf*> bufs() { return {&step_items, &step_rounds, &step_ctr, &step_fl, &round_items, &round_args}; }
};

// ===================================================================== context

static hipError_t walk_scratch_address(void** out);

extern "C" const char* gc_version(void) { return "gcharm-mi355x 0.1 (gfx950)"; }

extern "C" gc_status gc_init(int device, gc_alloc_fn alloc_fn, gc_free_fn free_fn, void* user, gc_ctx* out) {
  if (!out) return GC_E_INVAL;
  *out = nullptr;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return GC_E_INVAL;
  gc_ctx c = new gc_ctx_();
  c->device = device;
  c->hooks.alloc = alloc_fn;
  c->hooks.free = free_fn;
  c->hooks.user = user;
  c->walk_keep.h = &c->hooks;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete c;
    return GC_E_HIP;
  }
  hipDeviceProp_t p;
  e = hipGetDeviceProperties(&p, device);
  if (e != hipSuccess) {
    delete c;
    return GC_E_HIP;
  }
  c->n_cu = p.multiProcessorCount;
  e = walk_scratch_address(&c->walk_scratch);
  if (e != hipSuccess) {
    delete c;
    return GC_E_HIP;
  }
  *out = c;
  return GC_OK;
}

extern "C" gc_status gc_finalize(gc_ctx ctx) {
  if (!ctx) return GC_E_INVAL;
  ctx->walk_keep.release();
  delete ctx;
  return GC_OK;
}

extern "C" const char* gc_last_error(gc_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" gc_status gc_debug_inject_error(gc_ctx ctx, int hip_error) {
  if (!ctx || hip_error == 0) return GC_E_INVAL;
  ctx->injected = static_cast<hipError_t>(hip_error);
  return GC_OK;
}

extern "C" gc_status gc_debug_step_waits(gc_ctx ctx, uint32_t fail_spins, int32_t fail_round) {
  GC_ENTER(ctx);
  ctx->step_fail_spins = fail_spins;
  ctx->step_fail_round = fail_round < 0 ? -1 : fail_round;
  return GC_OK;
}

namespace {
// Reads device int32 words (each may be NULL) after waiting on the stream; returns the first nonzero
// word's index, or -1.
hipError_t first_set_word(const std::vector<const int32_t*>& words, hipStream_t s, int* hit) {
  *hit = -1;
  std::vector<int32_t> h(words.size(), 0);
  for (size_t k = 0; k < words.size(); ++k) {
    if (!words[k]) continue;
    hipError_t e = hipMemcpyAsync(&h[k], words[k], sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (size_t k = 0; k < words.size(); ++k)
    if (h[k] != 0) {
      *hit = (int)k;
      break;
    }
  return hipSuccess;
}
}  // namespace

extern "C" gc_status gc_zero_f32(gc_ctx ctx, float* dev, int64_t n, void* stream) {
  GC_ENTER(ctx);
  if (n < 0 || (n > 0 && !dev)) return set_err(ctx, GC_E_INVAL, "gc_zero_f32: bad buffer");
  GC_HIP(ctx, launch_fill_f32(dev, 0.f, n, S(stream)));
  return GC_OK;
}

// ===================================================================== pool

extern "C" gc_status gc_pool_create(gc_ctx ctx, int32_t n_ids, int32_t capacity, gc_pool* out) {
  GC_ENTER(ctx);
  if (!out || n_ids <= 0 || capacity <= 0) return set_err(ctx, GC_E_INVAL, "gc_pool_create: n_ids and capacity must be > 0");
  gc_pool p = new gc_pool_();
  p->ctx = ctx;
  p->n_ids = n_ids;
  p->cap = capacity;
  for (DevBuf* d : p->bufs()) d->h = &ctx->hooks;
  hipError_t e = p->rec.ensure(sizeof(float4) * (size_t)capacity);
  if (e == hipSuccess) e = p->slot_of.ensure(sizeof(int32_t) * (size_t)n_ids);
  if (e == hipSuccess) e = p->occ.ensure(sizeof(uint32_t) * (size_t)occ_words(capacity));
  if (e != hipSuccess) {
    p->rec.release(); p->slot_of.release(); p->occ.release();
    delete p;
    return set_err(ctx, GC_E_NOMEM, "gc_pool_create: %s", hipGetErrorString(e));
  }
  e = launch_fill_i32(p->slot_of.as<int32_t>(), -1, n_ids, nullptr);
  if (e == hipSuccess) e = launch_fill_i32(p->occ.as<int32_t>(), 0, occ_words(capacity), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    p->rec.release(); p->slot_of.release(); p->occ.release();
    delete p;
    return hip_fail(ctx, e, "gc_pool_create");
  }
  *out = p;
  return GC_OK;
}

extern "C" gc_status gc_pool_destroy(gc_pool pool) {
  if (!pool) return GC_E_INVAL;
  (void)hipDeviceSynchronize();
  for (DevBuf* d : pool->bufs()) d->release();
  pool->pin.release();
  pool->ev_pin.destroy();
  delete pool;
  return GC_OK;
}

// ---------------------------------------------------------------- host mirror of the chare table
// A host-source pool keeps the chare table on the host too.  The device's allocator is
// deterministic (the k-th missing id of a call takes the k-th lowest free slot), so every call the
// host makes can be replayed on the mirror in call order, and the host knows each request's missing
// set without reading the device.  Calls whose effect the host cannot see (a reorganisation from a
// device source, a graph launch) mark the mirror stale; it is then read back once, before the next
// host-staged call.

static void mirror_clear(gc_pool p) {
  p->m_slot_of.assign((size_t)p->n_ids, -1);
  p->m_free.assign(((size_t)p->cap + 63) / 64, ~0ull);
  if (p->cap % 64) p->m_free.back() = (1ull << (p->cap % 64)) - 1ull;
  p->m_nfree = p->cap;
  p->m_lo = 0;
  p->mirror_ok = true;
}

static void mirror_take_slot(gc_pool p, int32_t id, int32_t slot) {
  p->m_slot_of[id] = slot;
  uint64_t& w = p->m_free[(size_t)slot >> 6];
  const uint64_t bit = 1ull << (slot & 63);
  if (w & bit) {
    w &= ~bit;
    --p->m_nfree;
  }
}

static void mirror_free_id(gc_pool p, int32_t id) {
  const int32_t s = p->m_slot_of[id];
  if (s < 0) return;
  p->m_slot_of[id] = -1;
  uint64_t& w = p->m_free[(size_t)s >> 6];
  const uint64_t bit = 1ull << (s & 63);
  if (!(w & bit)) {
    w |= bit;
    ++p->m_nfree;
    p->m_lo = std::min(p->m_lo, (size_t)s >> 6);
  }
}

// The n lowest free slots, ascending, taken for ids[0, n) (fewer if the pool runs out: the rest
// get -1 and stay missing).
static void mirror_assign(gc_pool p, const int32_t* ids, int64_t n, int32_t* slots) {
  size_t w = p->m_lo;
  for (int64_t k = 0; k < n; ++k) {
    while (w < p->m_free.size() && !p->m_free[w]) ++w;
    if (w >= p->m_free.size()) {
      for (; k < n; ++k) slots[k] = -1;
      break;
    }
    const int32_t s = (int32_t)(w * 64 + (size_t)__builtin_ctzll(p->m_free[w]));
    p->m_free[w] &= p->m_free[w] - 1ull;
    --p->m_nfree;
    p->m_slot_of[ids[k]] = s;
    slots[k] = s;
  }
  p->m_lo = w;
}

// Reads the device's chare table and occupancy flags into the mirror (synchronises `s`).
static hipError_t mirror_sync(gc_pool p, hipStream_t s) {
  std::vector<uint32_t> occ((size_t)p->cap);
  p->m_slot_of.resize((size_t)p->n_ids);
  hipError_t e = hipMemcpyAsync(p->m_slot_of.data(), p->slot_of.p, sizeof(int32_t) * (size_t)p->n_ids,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(occ.data(), p->occ.p, sizeof(uint32_t) * (size_t)p->cap, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  p->m_free.assign(((size_t)p->cap + 63) / 64, 0ull);
  p->m_nfree = 0;
  for (int32_t k = 0; k < p->cap; ++k)
    if (occ[k] == 0u) {
      p->m_free[(size_t)k >> 6] |= 1ull << (k & 63);
      ++p->m_nfree;
    }
  p->m_lo = 0;
  p->mirror_ok = true;
  return hipSuccess;
}

// Copies n device int32 values to the host (synchronises `s`).
static hipError_t read_ids(const int32_t* dev, int32_t n, std::vector<int32_t>& out, hipStream_t s) {
  out.resize((size_t)std::max(n, 0));
  if (n <= 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(out.data(), dev, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s);
  return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

extern "C" gc_status gc_pool_set_source(gc_pool pool, const void* records) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (!records) return set_err(pool->ctx, GC_E_INVAL, "gc_pool_set_source: NULL records");
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, records);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(pool->ctx, GC_E_INVAL, "gc_pool_set_source: pointer is neither device memory nor pinned host memory");
  }
  pool->src_device = (at.type == hipMemoryTypeDevice);
  pool->host_src = nullptr;
  if (at.type == hipMemoryTypeHost) {
    // pinned host memory: use its device-visible address
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, const_cast<void*>(records), 0) != hipSuccess || !dp) {
      (void)hipGetLastError();
      return set_err(pool->ctx, GC_E_INVAL, "gc_pool_set_source: host memory is not device-accessible (use hipHostMalloc)");
    }
    pool->src = static_cast<const float4*>(dp);
  } else if (at.type == hipMemoryTypeDevice) {
    pool->src = static_cast<const float4*>(records);
  } else {
    return set_err(pool->ctx, GC_E_INVAL, "gc_pool_set_source: unsupported memory type");
  }
  return GC_OK;
}

extern "C" gc_status gc_pool_set_host_source(gc_pool pool, const void* records) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (!records) return set_err(pool->ctx, GC_E_INVAL, "gc_pool_set_host_source: NULL records");
  pool->host_src = static_cast<const float4*>(records);
  pool->src = nullptr;
  pool->src_device = false;
  pool->mirror_ok = false;  // read back before the first host-staged call
  return GC_OK;
}

extern "C" gc_status gc_pool_place(gc_pool pool, const int32_t* ids_dev, const int32_t* slots_dev, int32_t n,
                                   void* stream) {
  if (!pool) return GC_E_INVAL;
  gc_ctx c = pool->ctx;
  GC_ENTER(c);
  if (n < 0 || (n > 0 && (!ids_dev || !slots_dev))) return set_err(c, GC_E_INVAL, "gc_pool_place: bad arrays");
  if (n > 0 && !pool->src && !pool->host_src) return set_err(c, GC_E_STATE, "gc_pool_place: no source set");
  if (n == 0) return GC_OK;
  hipStream_t s = S(stream);
  if (!pool->host_src) {
    pool->mirror_ok = false;
    GC_HIP(c, launch_place(ids_dev, slots_dev, n, pool->src, false, pool->rec.as<float4>(),
                           pool->slot_of.as<int32_t>(), pool->occ.as<uint32_t>(), s));
    return GC_OK;
  }
  // host source: the host reads the fixture, packs the records and copies them in
  std::vector<int32_t> ids, slots;
  GC_HIP(c, read_ids(ids_dev, n, ids, s));
  GC_HIP(c, read_ids(slots_dev, n, slots, s));
  for (int32_t k = 0; k < n; ++k)
    if (ids[k] < 0 || ids[k] >= pool->n_ids || slots[k] < 0 || slots[k] >= pool->cap)
      return set_err(c, GC_E_INVAL, "gc_pool_place: id %d or slot %d out of range", ids[k], slots[k]);
  if (!pool->mirror_ok) GC_HIP(c, mirror_sync(pool, s));
  GC_HIP(c, pool->ev_pin.sync());
  if (pool->pin.ensure(sizeof(float4) * (size_t)n) != hipSuccess || pool->tmp.ensure(sizeof(float4) * (size_t)n) != hipSuccess)
    return set_err(c, GC_E_NOMEM, "gc_pool_place: staging buffers");
  float4* pin = pool->pin.as<float4>();
  for (int32_t k = 0; k < n; ++k) pin[k] = pool->host_src[ids[k]];
  GC_HIP(c, hipMemcpyAsync(pool->tmp.p, pin, sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, s));
  GC_HIP(c, pool->ev_pin.record(s));
  GC_HIP(c, launch_place(ids_dev, slots_dev, n, pool->tmp.as<float4>(), true, pool->rec.as<float4>(),
                         pool->slot_of.as<int32_t>(), pool->occ.as<uint32_t>(), s));
  for (int32_t k = 0; k < n; ++k) mirror_take_slot(pool, ids[k], slots[k]);
  return GC_OK;
}

static hipError_t pool_reset_async(gc_pool pool, hipStream_t s) {
  return launch_pool_reset(pool->slot_of.as<int32_t>(), pool->n_ids, pool->occ.as<uint32_t>(), pool->cap, s);
}

extern "C" gc_status gc_pool_reset(gc_pool pool, void* stream) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  GC_HIP(pool->ctx, pool_reset_async(pool, S(stream)));
  if (pool->host_src) mirror_clear(pool);
  else pool->mirror_ok = false;
  return GC_OK;
}

extern "C" gc_status gc_pool_query_mirror(gc_pool pool, int32_t* slot_of_host, void* stream) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (!slot_of_host) return set_err(pool->ctx, GC_E_INVAL, "gc_pool_query_mirror: NULL output");
  if (!pool->host_src) return set_err(pool->ctx, GC_E_STATE, "gc_pool_query_mirror: the pool has no host source");
  if (!pool->mirror_ok) GC_HIP(pool->ctx, mirror_sync(pool, S(stream)));
  std::memcpy(slot_of_host, pool->m_slot_of.data(), sizeof(int32_t) * (size_t)pool->n_ids);
  return GC_OK;
}

extern "C" gc_status gc_pool_query(gc_pool pool, int32_t* slot_of_host, void* stream) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (!slot_of_host) return set_err(pool->ctx, GC_E_INVAL, "gc_pool_query: NULL output");
  GC_HIP(pool->ctx, hipMemcpyAsync(slot_of_host, pool->slot_of.p, sizeof(int32_t) * (size_t)pool->n_ids,
                                   hipMemcpyDeviceToHost, S(stream)));
  GC_HIP(pool->ctx, hipStreamSynchronize(S(stream)));
  return GC_OK;
}

extern "C" gc_status gc_pool_device_ptrs(gc_pool pool, void** records, int32_t** slot_of) {
  if (!pool) return GC_E_INVAL;
  if (records) *records = pool->rec.p;
  if (slot_of) *slot_of = pool->slot_of.as<int32_t>();
  return GC_OK;
}

// ===================================================================== batch

extern "C" gc_status gc_batch_create(gc_ctx ctx, int32_t kind, int32_t n_ids, gc_batch* out) {
  GC_ENTER(ctx);
  if (!out || n_ids <= 0 || (kind != GC_KIND_GRAV && kind != GC_KIND_LJ))
    return set_err(ctx, GC_E_INVAL, "gc_batch_create: bad kind or n_ids");
  gc_batch b = new gc_batch_();
  b->ctx = ctx;
  b->kind = kind;
  b->n_ids = n_ids;
  for (DevBuf* d : b->bufs()) d->h = &ctx->hooks;
  *out = b;
  return GC_OK;
}

extern "C" gc_status gc_batch_destroy(gc_batch b) {
  if (!b) return GC_E_INVAL;
  (void)hipDeviceSynchronize();
  for (DevBuf* d : b->bufs()) d->release();
  b->pin.release();
  b->ev_copy.destroy();
  b->ev_use.destroy();
  delete b;
  return GC_OK;
}

extern "C" gc_status gc_batch_reset(gc_batch b) {
  if (!b) return GC_E_INVAL;
  GC_ENTER(b->ctx);
  b->tasks.clear();
  b->ranges.clear();
  b->nodes.clear();
  b->n_direct = b->n_targets = 0;
  b->max_node = -1;
  b->committed = false;
  b->ranks_ready = false;
  b->hU.clear();
  b->u = 0;
  b->mode = -1;
  b->pool = nullptr;
  b->host_staged = false;
  b->h_missing.clear();
  b->h_mslot.clear();
  b->nt = b->nr = b->nn = 0;
  b->dev_sub = false;
  b->host_lists = true;
  return GC_OK;
}

extern "C" gc_status gc_submit_tasks(gc_batch b, const gc_task* tasks, int32_t n_tasks, const int32_t* j_ranges,
                                     int32_t n_ranges, const int32_t* node_idx, int32_t n_node_refs) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (b->dev_sub) return set_err(c, GC_E_STATE, "gc_submit_tasks: the batch holds a device submission (reset it first)");
  if (n_tasks < 0 || n_ranges < 0 || n_node_refs < 0) return set_err(c, GC_E_INVAL, "gc_submit_tasks: negative count");
  if ((n_tasks && !tasks) || (n_ranges && !j_ranges) || (n_node_refs && !node_idx))
    return set_err(c, GC_E_INVAL, "gc_submit_tasks: NULL array with nonzero count");
  int64_t add_direct = 0, add_targets = 0;
  for (int32_t r = 0; r < n_ranges; ++r) {
    int64_t s = j_ranges[2 * r], n = j_ranges[2 * r + 1];
    if (s < 0 || n < 0 || s + n > b->n_ids)
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: range %d (%lld, %lld) outside [0, %d)", r, (long long)s,
                     (long long)n, b->n_ids);
  }
  int32_t max_node = b->max_node;
  for (int32_t k = 0; k < n_node_refs; ++k) {
    if (node_idx[k] < 0) return set_err(c, GC_E_INVAL, "gc_submit_tasks: negative node index at %d", k);
    max_node = std::max(max_node, node_idx[k]);
  }
  std::vector<std::pair<int32_t, int32_t>> tr;  // one task's nonempty direct ranges, for the overlap test
  for (int32_t t = 0; t < n_tasks; ++t) {
    const gc_task& tk = tasks[t];
    if (tk.i_count < 0 || tk.i_begin < 0 || (int64_t)tk.i_begin + tk.i_count > b->n_ids)
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: task %d targets outside [0, %d)", t, b->n_ids);
    if (tk.j_nranges < 0 || tk.j_first < 0 || (int64_t)tk.j_first + tk.j_nranges > n_ranges)
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: task %d range slice outside the given ranges", t);
    if (tk.n_count < 0 || tk.n_first < 0 || (int64_t)tk.n_first + tk.n_count > n_node_refs)
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: task %d node slice outside the given node refs", t);
    if (b->kind == GC_KIND_LJ && (tk.j_nranges != 1 || tk.n_count != 0))
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: Lennard-Jones task %d needs exactly one j range and no nodes", t);
    if (b->kind == GC_KIND_GRAV && (tk.flags != 0 || tk.shift[0] != 0.f || tk.shift[1] != 0.f || tk.shift[2] != 0.f))
      return set_err(c, GC_E_INVAL, "gc_submit_tasks: gravity task %d has flags or a shift", t);
    if (b->kind == GC_KIND_LJ && (tk.flags & GC_TASK_SELF)) {
      const int32_t* g = j_ranges + 2 * tk.j_first;
      if (g[0] != tk.i_begin || g[1] != tk.i_count)
        return set_err(c, GC_E_INVAL, "gc_submit_tasks: self task %d must use its target range as j range", t);
    }
    for (int32_t r = 0; r < tk.j_nranges; ++r) add_direct += j_ranges[2 * (tk.j_first + r) + 1];
    add_targets += tk.i_count;
    // a source listed twice would be counted twice: the direct ranges of a task must not overlap
    if (tk.j_nranges > 1) {
      tr.clear();
      for (int32_t r = 0; r < tk.j_nranges; ++r) {
        const int32_t* g = j_ranges + 2 * (tk.j_first + r);
        if (g[1] > 0) tr.emplace_back(g[0], g[1]);
      }
      std::sort(tr.begin(), tr.end());
      for (size_t q = 1; q < tr.size(); ++q)
        if ((int64_t)tr[q - 1].first + tr[q - 1].second > tr[q].first)
          return set_err(c, GC_E_INVAL, "gc_submit_tasks: task %d has overlapping direct ranges at ids %d and %d", t,
                         tr[q - 1].first, tr[q].first);
    }
  }
  if (b->n_direct + add_direct > INT32_MAX || b->n_targets + add_targets > INT32_MAX ||
      (int64_t)b->tasks.size() + n_tasks > INT32_MAX || (int64_t)b->ranges.size() / 2 + n_ranges > INT32_MAX)
    return set_err(c, GC_E_INVAL, "gc_submit_tasks: batch exceeds 2^31 entries");
  const int32_t r0 = (int32_t)(b->ranges.size() / 2), n0 = (int32_t)b->nodes.size();
  for (int32_t t = 0; t < n_tasks; ++t) {
    gc_task tk = tasks[t];
    tk.j_first += r0;
    tk.n_first += n0;
    b->tasks.push_back(tk);
  }
  b->ranges.insert(b->ranges.end(), j_ranges, j_ranges + 2 * (size_t)n_ranges);
  b->nodes.insert(b->nodes.end(), node_idx, node_idx + n_node_refs);
  b->n_direct += add_direct;
  b->n_targets += add_targets;
  b->nt = (int32_t)b->tasks.size();
  b->nr = (int32_t)(b->ranges.size() / 2);
  b->nn = (int32_t)b->nodes.size();
  b->max_node = max_node;
  b->committed = false;
  b->ranks_ready = false;
  b->mode = -1;
  return GC_OK;
}

extern "C" gc_status gc_batch_sizes(gc_batch b, int64_t* out5) {
  if (!b || !out5) return GC_E_INVAL;
  out5[0] = b->nt;
  out5[1] = b->nr;
  out5[2] = b->nn;
  out5[3] = b->n_direct;
  out5[4] = b->n_targets;
  return GC_OK;
}

extern "C" gc_status gc_batch_status(gc_batch b, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  const int32_t* wait_word = b->state.p ? b->state.as<int32_t>() + GC_STATE_ERR : nullptr;
  const int32_t* node_word = b->stat.p ? b->stat.as<int32_t>() : nullptr;
  int hit = -1;
  GC_HIP(c, first_set_word({wait_word, node_word}, S(stream), &hit));
  if (hit == 0) return set_err(c, GC_E_HIP, "gc_batch_status: a bounded wait of a reorganisation gave up");
  if (hit == 1) return set_err(c, GC_E_INVAL, "gc_batch_status: a backward call met node ranges outside [0, n_ids)");
  return GC_OK;
}

// ---------------------------------------------------------------- device submission and commit

extern "C" gc_status gc_submit_tasks_device(gc_batch b, const gc_task* tasks_dev, int32_t n_tasks,
                                            const int32_t* j_ranges_dev, int32_t n_ranges,
                                            const int32_t* node_idx_dev, int32_t n_node_refs, int32_t n_nodes,
                                            void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (b->kind != GC_KIND_GRAV) return set_err(c, GC_E_UNSUPPORTED, "gc_submit_tasks_device: gravity batches only");
  if (b->nt || b->nr || b->nn || b->dev_sub)
    return set_err(c, GC_E_STATE, "gc_submit_tasks_device: the batch already holds tasks (reset it first)");
  if (n_tasks < 0 || n_ranges < 0 || n_node_refs < 0 || n_nodes < 0)
    return set_err(c, GC_E_INVAL, "gc_submit_tasks_device: negative count");
  if ((n_tasks && !tasks_dev) || (n_ranges && !j_ranges_dev) || (n_node_refs && !node_idx_dev))
    return set_err(c, GC_E_INVAL, "gc_submit_tasks_device: NULL array with nonzero count");
  hipStream_t s = S(stream);
  hipError_t e = b->d_tasks.ensure(sizeof(gc_task) * (size_t)std::max(n_tasks, 1));
  if (e == hipSuccess) e = b->d_ranges.ensure(sizeof(int32_t) * 2 * (size_t)std::max(n_ranges, 1));
  if (e == hipSuccess) e = b->d_nodes.ensure(sizeof(int32_t) * (size_t)std::max(n_node_refs, 1));
  if (e != hipSuccess) return set_err(c, GC_E_NOMEM, "gc_submit_tasks_device: %s", hipGetErrorString(e));
  if (n_tasks)
    GC_HIP(c, hipMemcpyAsync(b->d_tasks.p, tasks_dev, sizeof(gc_task) * (size_t)n_tasks, hipMemcpyDeviceToDevice, s));
  if (n_ranges)
    GC_HIP(c, hipMemcpyAsync(b->d_ranges.p, j_ranges_dev, sizeof(int32_t) * 2 * (size_t)n_ranges,
                             hipMemcpyDeviceToDevice, s));
  if (n_node_refs)
    GC_HIP(c, hipMemcpyAsync(b->d_nodes.p, node_idx_dev, sizeof(int32_t) * (size_t)n_node_refs,
                             hipMemcpyDeviceToDevice, s));
  b->nt = n_tasks;
  b->nr = n_ranges;
  b->nn = n_node_refs;
  b->dev_n_nodes = n_nodes;
  b->dev_sub = true;
  b->host_lists = false;
  b->committed = false;
  b->mode = -1;
  return GC_OK;
}

extern "C" gc_status gc_walk_tasks(gc_ctx c, int32_t n_buckets, int32_t b0, int32_t b1, const int32_t* bucket_node_dev,
                                   int32_t n_nodes, const int32_t* node_range_dev, const int32_t* n_first_dev,
                                   const int32_t* r_first_dev, gc_task* tasks_dev, void* stream) {
  GC_ENTER(c);
  if (b0 < 0 || b1 < b0 || b1 > n_buckets || n_nodes < 0)
    return set_err(c, GC_E_INVAL, "gc_walk_tasks: bucket range [%d, %d) not inside [0, %d), or n_nodes < 0", b0, b1,
                   n_buckets);
  if (b1 > b0 && (!bucket_node_dev || !node_range_dev || !n_first_dev || !r_first_dev || !tasks_dev))
    return set_err(c, GC_E_INVAL, "gc_walk_tasks: NULL array");
  GC_HIP(c, launch_walk_tasks(b0, b1, bucket_node_dev, n_nodes, node_range_dev, n_first_dev, r_first_dev, tasks_dev,
                              S(stream)));
  return GC_OK;
}

// The whole commit of a device submission runs on the device; the host reads back eight totals.
static gc_status commit_device(gc_batch b, hipStream_t s) {
  gc_ctx c = b->ctx;
  const int32_t T = b->nt, n = b->n_ids;
  const int nb = dc_id_blocks(n);
  hipError_t e = b->dc_dc.ensure(sizeof(int32_t) * (size_t)std::max(T, 1));
  if (e == hipSuccess) e = b->dc_cost.ensure(sizeof(int64_t) * (size_t)std::max(T, 1));
  if (e == hipSuccess) e = b->dc_diff.ensure(sizeof(int32_t) * 2 * ((size_t)n + 1));
  if (e == hipSuccess) e = b->dc_bs.ensure(sizeof(int32_t) * 2 * (size_t)nb);
  if (e == hipSuccess) e = b->dc_ns.ensure(sizeof(int32_t) * (size_t)nb);
  if (e == hipSuccess) e = b->dc_tot.ensure(sizeof(int64_t) * kDcTot);
  if (e == hipSuccess) e = b->d_U.ensure(sizeof(int32_t) * (size_t)union_padded(n));
  if (e == hipSuccess) e = b->d_pos.ensure(sizeof(int32_t) * (size_t)n);
  if (e == hipSuccess) e = b->pranges.ensure(sizeof(int32_t) * 2 * (size_t)std::max(b->nr, 1));
  if (e == hipSuccess) e = b->pibeg.ensure(sizeof(int32_t) * (size_t)std::max(T, 1));
  if (e == hipSuccess) e = b->d_ioff.ensure(sizeof(int32_t) * (size_t)std::max(T, 1));
  if (e == hipSuccess) e = b->d_joff.ensure(sizeof(int32_t) * ((size_t)T + 1));
  if (e == hipSuccess) e = b->d_order.ensure(sizeof(int32_t) * (size_t)std::max(T, 1));
  if (e == hipSuccess) e = b->stat.ensure(sizeof(int32_t) * 4);
  if (e != hipSuccess) return set_err(c, GC_E_NOMEM, "gc_batch_commit: %s", hipGetErrorString(e));
  GC_HIP(c, launch_fill_i32(b->dc_diff.as<int32_t>(), 0, 2 * ((int64_t)n + 1), s));
  GC_HIP(c, launch_fill_i32(b->dc_tot.as<int32_t>(), 0, 2 * kDcTot, s));
  GC_HIP(c, launch_fill_i32(b->d_U.as<int32_t>(), 0, union_padded(n), s));
  GC_HIP(c, launch_fill_i32(b->stat.as<int32_t>(), 0, 4, s));
  DevCommitArgs a{};
  a.tasks = b->d_tasks.as<gc_task>();
  a.n_tasks = T;
  a.ranges = b->d_ranges.as<int2>();
  a.n_ranges = b->nr;
  a.nodes = b->d_nodes.as<int32_t>();
  a.n_node_refs = b->nn;
  a.n_nodes = b->dev_n_nodes;
  a.n_ids = n;
  a.dc = b->dc_dc.as<int32_t>();
  a.cost = b->dc_cost.as<int64_t>();
  a.diff = b->dc_diff.as<int32_t>();
  a.bs = b->dc_bs.as<int32_t>();
  a.ns = b->dc_ns.as<int32_t>();
  a.U = b->d_U.as<int32_t>();
  a.pos = b->d_pos.as<int32_t>();
  a.pranges = b->pranges.as<int2>();
  a.pibeg = b->pibeg.as<int32_t>();
  a.ioff = b->d_ioff.as<int32_t>();
  a.joff = b->d_joff.as<int32_t>();
  a.order = b->d_order.as<int32_t>();
  a.tot = b->dc_tot.as<int64_t>();
  GC_HIP(c, launch_dev_commit(a, s));
  int64_t tot[kDcTot];
  GC_HIP(c, hipMemcpyAsync(tot, b->dc_tot.p, sizeof tot, hipMemcpyDeviceToHost, s));
  GC_HIP(c, hipStreamSynchronize(s));
  if (tot[kDcBad] || tot[kDcBadTargets]) {
    return set_err(c, GC_E_INVAL,
                   "gc_batch_commit: device submission with %lld task(s) outside the contract (ids, slices, "
                   "ranges not ascending and disjoint, node indices) and %lld id(s) targeted by two tasks",
                   (long long)tot[kDcBad], (long long)tot[kDcBadTargets]);
  }
  if (tot[kDcDirect] > INT32_MAX || tot[kDcTargets] > INT32_MAX)
    return set_err(c, GC_E_INVAL, "gc_batch_commit: batch exceeds 2^31 entries");
  b->u = (int32_t)tot[kDcUnion];
  b->n_direct = tot[kDcDirect];
  b->n_targets = tot[kDcTargets];
  b->max_direct = (int32_t)tot[kDcMaxDirect];
  b->max_node = b->nn ? (int32_t)tot[kDcMaxNode] : -1;
  b->n_runs = 0;
  b->lj_gather = b->lj_cover = false;
  b->n_ljtgt = 0;
  b->host_lists = false;
  b->committed = true;
  b->ranks_ready = false;
  b->adj_nodes = -1;
  b->mode = -1;
  return GC_OK;
}

// The host copies of a device-committed batch's tasks, lists, union and launch order, read from the
// device when a host-side step first needs them (synchronises `s`).
static gc_status need_host_lists(gc_batch b, hipStream_t s) {
  if (b->host_lists) return GC_OK;
  gc_ctx c = b->ctx;
  b->tasks.resize((size_t)b->nt);
  b->ranges.resize(2 * (size_t)b->nr);
  b->nodes.resize((size_t)b->nn);
  b->hU.resize((size_t)b->u);
  b->h_order.resize((size_t)b->nt);
  b->h_pibeg.resize((size_t)b->nt);
  auto dn = [&](void* dst, const DevBuf& src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src.p, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
  };
  GC_HIP(c, dn(b->tasks.data(), b->d_tasks, sizeof(gc_task) * b->tasks.size()));
  GC_HIP(c, dn(b->ranges.data(), b->d_ranges, sizeof(int32_t) * b->ranges.size()));
  GC_HIP(c, dn(b->nodes.data(), b->d_nodes, sizeof(int32_t) * b->nodes.size()));
  GC_HIP(c, dn(b->hU.data(), b->d_U, sizeof(int32_t) * b->hU.size()));
  GC_HIP(c, dn(b->h_order.data(), b->d_order, sizeof(int32_t) * b->h_order.size()));
  GC_HIP(c, dn(b->h_pibeg.data(), b->pibeg, sizeof(int32_t) * b->h_pibeg.size()));
  GC_HIP(c, hipStreamSynchronize(s));
  b->host_lists = true;
  return GC_OK;
}

extern "C" gc_status gc_batch_commit(gc_batch b, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (b->committed) return GC_OK;
  if (b->dev_sub) return commit_device(b, S(stream));
  const int32_t T = (int32_t)b->tasks.size();
  const int32_t R = (int32_t)(b->ranges.size() / 2);
  // targets written by at most one gravity task
  if (b->kind == GC_KIND_GRAV) {
    std::vector<uint8_t> hit((size_t)b->n_ids, 0);
    for (int32_t t = 0; t < T; ++t)
      for (int32_t i = b->tasks[t].i_begin; i < b->tasks[t].i_begin + b->tasks[t].i_count; ++i) {
        if (hit[i]) return set_err(c, GC_E_INVAL, "gc_batch_commit: id %d is the target of two gravity tasks", i);
        hit[i] = 1;
      }
  }
  std::vector<int32_t> ioff(T > 0 ? T : 1), joff((size_t)T + 1, 0);
  int64_t io = 0;
  int32_t maxd = 0;
  std::vector<int64_t> cost(T);
  for (int32_t t = 0; t < T; ++t) {
    const gc_task& tk = b->tasks[t];
    ioff[t] = (int32_t)io;
    io += tk.i_count;
    int64_t d = 0;
    for (int32_t r = 0; r < tk.j_nranges; ++r) d += b->ranges[2 * (tk.j_first + r) + 1];
    joff[t + 1] = joff[t] + (int32_t)d;
    maxd = std::max<int32_t>(maxd, (int32_t)d);
    cost[t] = (int64_t)tk.i_count * (b->kind == GC_KIND_GRAV ? (31 * (int64_t)tk.n_count + 12 * d) : d);
  }
  b->max_direct = maxd;
  // the union U: sorted distinct ids over all target and direct ranges (the merged intervals,
  // expanded), and each range's first position in it (a range is contiguous in U)
  std::vector<std::pair<int32_t, int32_t>> mk;
  mk.reserve((size_t)T + R);
  for (int32_t t = 0; t < T; ++t)
    if (b->tasks[t].i_count > 0) mk.emplace_back(b->tasks[t].i_begin, b->tasks[t].i_begin + b->tasks[t].i_count);
  for (int32_t r = 0; r < R; ++r)
    if (b->ranges[2 * r + 1] > 0) mk.emplace_back(b->ranges[2 * r], b->ranges[2 * r] + b->ranges[2 * r + 1]);
  std::sort(mk.begin(), mk.end());
  b->hU.clear();
  {
    int64_t covered = -1;  // ids below this are already in U
    for (auto& m : mk) {
      for (int64_t id = std::max<int64_t>(m.first, covered); id < m.second; ++id) b->hU.push_back((int32_t)id);
      covered = std::max<int64_t>(covered, m.second);
    }
  }
  b->u = (int32_t)b->hU.size();
  auto upos = [&](int32_t id) -> int32_t {
    return (int32_t)(std::lower_bound(b->hU.begin(), b->hU.end(), id) - b->hU.begin());
  };
  std::vector<int32_t> pr((size_t)2 * R), pib(T > 0 ? T : 1, 0);
  for (int32_t r = 0; r < R; ++r) {
    pr[2 * r] = b->ranges[2 * r + 1] > 0 ? upos(b->ranges[2 * r]) : 0;
    pr[2 * r + 1] = b->ranges[2 * r + 1];
  }
  for (int32_t t = 0; t < T; ++t) pib[t] = b->tasks[t].i_count > 0 ? upos(b->tasks[t].i_begin) : 0;
  std::vector<int32_t> upad((size_t)union_padded(b->u), 0);
  std::copy(b->hU.begin(), b->hU.end(), upad.begin());
  // task order: longest first within each run of kLptChunk consecutive tasks.  Within a run the
  // long tasks start first (the launch ends with short ones); runs stay in submission order, so
  // the tasks in flight at one time come from neighbouring buckets (or from one instance of a
  // batch of instances) and share node and particle data in the caches
  std::vector<int32_t> order(T > 0 ? T : 1);
  std::iota(order.begin(), order.begin() + T, 0);
  for (int32_t c0 = 0; c0 < T; c0 += kLptChunk)
    std::stable_sort(order.begin() + c0, order.begin() + std::min<int32_t>(T, c0 + kLptChunk),
                     [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });

  // runs of consecutive tasks sharing one target range (processed by one wavefront for LJ)
  std::vector<int32_t> runs;
  runs.reserve((size_t)T + 1);
  for (int32_t t = 0; t < T; ++t)
    if (t == 0 || b->tasks[t].i_begin != b->tasks[t - 1].i_begin || b->tasks[t].i_count != b->tasks[t - 1].i_count)
      runs.push_back(t);
  runs.push_back(T);
  b->n_runs = (int32_t)runs.size() - 1;
  // Lennard-Jones gather form: every task's i range (side 0) and, unless it is the cell's own
  // self task, its j range (side 1) is a target range; ranges of equal extent merge, and the form
  // needs the distinct ones disjoint (each id then has one wavefront that writes it)
  std::vector<int32_t> ljtgt, ljent;
  b->lj_gather = false;
  b->lj_cover = false;
  b->n_ljtgt = 0;
  if (b->kind == GC_KIND_LJ) {
    struct Side { int32_t begin, count, task, side; };
    std::vector<Side> sides;
    sides.reserve((size_t)2 * T);
    for (int32_t t = 0; t < T; ++t) {
      const gc_task& tk = b->tasks[t];
      const int32_t jb = b->ranges[2 * tk.j_first], jn = b->ranges[2 * tk.j_first + 1];
      if (tk.i_count > 0 && jn > 0) {
        sides.push_back({tk.i_begin, tk.i_count, t, 0});
        if (!(tk.flags & GC_TASK_SELF)) sides.push_back({jb, jn, t, 1});
      }
    }
    std::sort(sides.begin(), sides.end(), [](const Side& x, const Side& y) {
      if (x.begin != y.begin) return x.begin < y.begin;
      if (x.count != y.count) return x.count < y.count;
      return 2 * (int64_t)x.task + x.side < 2 * (int64_t)y.task + y.side;
    });
    bool ok = true;
    int64_t covered = 0, prev_end = 0;
    for (size_t k = 0; k < sides.size();) {
      size_t e = k;
      while (e < sides.size() && sides[e].begin == sides[k].begin && sides[e].count == sides[k].count) ++e;
      if (sides[k].begin < prev_end) { ok = false; break; }
      ljtgt.insert(ljtgt.end(), {sides[k].begin, sides[k].count, (int32_t)ljent.size(), (int32_t)(e - k)});
      for (size_t q = k; q < e; ++q) ljent.push_back(2 * sides[q].task + sides[q].side);
      prev_end = (int64_t)sides[k].begin + sides[k].count;
      covered += sides[k].count;
      k = e;
    }
    if (ok) {
      b->lj_gather = true;
      b->lj_cover = covered == b->n_ids;
      b->n_ljtgt = (int32_t)(ljtgt.size() / 4);
    }
  }
  hipStream_t s = S(stream);
  hipError_t e = hipSuccess;
  auto up = [&](DevBuf& d, const void* src, size_t bytes) {
    if (e != hipSuccess) return;
    e = d.ensure(bytes);
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, s);
  };
  up(b->d_tasks, b->tasks.data(), sizeof(gc_task) * (size_t)T);
  up(b->d_ranges, b->ranges.data(), sizeof(int32_t) * b->ranges.size());
  up(b->d_nodes, b->nodes.data(), sizeof(int32_t) * b->nodes.size());
  up(b->d_U, upad.data(), sizeof(int32_t) * upad.size());
  up(b->pranges, pr.data(), sizeof(int32_t) * pr.size());
  up(b->pibeg, pib.data(), sizeof(int32_t) * pib.size());
  up(b->d_ioff, ioff.data(), sizeof(int32_t) * ioff.size());
  up(b->d_joff, joff.data(), sizeof(int32_t) * joff.size());
  up(b->d_order, order.data(), sizeof(int32_t) * order.size());
  up(b->d_runs, runs.data(), sizeof(int32_t) * runs.size());
  if (b->lj_gather) {
    up(b->d_ljtgt, ljtgt.data(), sizeof(int32_t) * ljtgt.size());
    up(b->d_ljent, ljent.data(), sizeof(int32_t) * ljent.size());
  }
  if (e == hipSuccess) e = b->stat.ensure(sizeof(int32_t) * 4);
  if (e == hipSuccess) e = launch_fill_i32(b->stat.as<int32_t>(), 0, 4, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host vectors must outlive the copies
  if (e != hipSuccess) return hip_fail(c, e, "gc_batch_commit");
  order.resize((size_t)T);
  pib.resize((size_t)T);
  b->h_order = std::move(order);
  b->h_pibeg = std::move(pib);
  b->committed = true;
  b->ranks_ready = false;
  b->adj_nodes = -1;
  b->mode = -1;
  return GC_OK;
}

// Reorganisation state (int32 words): [0, 8) counts read by the host (GC_STATE_*), then the
// ticket and completion counters, the current call tag, the free-slot total and the look-back
// words of both chains.  Tags make the words and the free-slot list self-invalidating; both are
// zeroed whenever either is (re)allocated so that no stale entry can carry a future tag.
static bool lists_mode(int32_t mode) { return mode == GC_REORG_INDIRECT || mode == GC_REORG_SORTED; }

// Visit indices of the gravity adjoint.  Node visits (entries of the node lists, in list order) are
// grouped by node by a counting sort, keeping visit order within a node, and each node's run is cut
// into chunks of at most kVisitChunk; direct visits (the tasks' flat direct positions, tasks in order)
// are grouped the same way by source id.  Node ids must lie in [0, n_nodes).
static gc_status build_adj_index(gc_batch b, int32_t n_nodes, hipStream_t s) {
  gc_ctx c = b->ctx;
  gc_status hs = need_host_lists(b, s);
  if (hs != GC_OK) return hs;
  const int64_t nv = (int64_t)b->nodes.size();
  std::vector<int32_t> nstart((size_t)n_nodes + 1, 0);
  for (int64_t v = 0; v < nv; ++v) {
    const int32_t nd = b->nodes[v];
    if (nd >= n_nodes) return set_err(c, GC_E_INVAL, "gc_backward: node index %d at list entry %lld >= n_nodes %d",
                                      nd, (long long)v, n_nodes);
    ++nstart[(size_t)nd + 1];
  }
  for (int32_t k = 0; k < n_nodes; ++k) nstart[k + 1] += nstart[k];
  std::vector<int32_t> nvis((size_t)std::max<int64_t>(nv, 1));
  {
    std::vector<int32_t> fill(nstart.begin(), nstart.end() - 1);
    for (int64_t v = 0; v < nv; ++v) nvis[fill[b->nodes[v]]++] = (int32_t)v;
  }
  std::vector<int32_t> chunks, chunk_first((size_t)n_nodes + 1);
  for (int32_t k = 0; k < n_nodes; ++k) {
    chunk_first[k] = (int32_t)(chunks.size() / 2);
    for (int32_t c0 = nstart[k]; c0 < nstart[k + 1]; c0 += kVisitChunk) {
      chunks.push_back(c0);
      chunks.push_back(std::min(c0 + kVisitChunk, nstart[k + 1]));
    }
  }
  chunk_first[n_nodes] = (int32_t)(chunks.size() / 2);
  if (chunks.empty()) chunks.assign(2, 0);
  const int32_t n_ids = b->n_ids;
  std::vector<int32_t> dstart((size_t)n_ids + 1, 0), dvis((size_t)std::max<int64_t>(b->n_direct, 1)),
      dkey((size_t)std::max<int64_t>(b->n_direct, 1));
  for (const gc_task& tk : b->tasks)
    for (int32_t r = 0; r < tk.j_nranges; ++r) {
      const int32_t g0 = b->ranges[2 * (tk.j_first + r)], gn = b->ranges[2 * (tk.j_first + r) + 1];
      for (int32_t k = 0; k < gn; ++k) ++dstart[(size_t)g0 + k + 1];
    }
  for (int32_t k = 0; k < n_ids; ++k) dstart[k + 1] += dstart[k];
  {
    std::vector<int32_t> fill(dstart.begin(), dstart.end() - 1);
    int32_t v = 0;
    for (const gc_task& tk : b->tasks)
      for (int32_t r = 0; r < tk.j_nranges; ++r) {
        const int32_t g0 = b->ranges[2 * (tk.j_first + r)], gn = b->ranges[2 * (tk.j_first + r) + 1];
        for (int32_t k = 0; k < gn; ++k) {
          dkey[fill[g0 + k]] = g0 + k;
          dvis[fill[g0 + k]++] = v++;
        }
      }
  }
  const int nq = 3;  // room for the quadrupole records, so one build serves both orders
  hipError_t e = b->vnode.ensure(sizeof(float4) * nq * (size_t)std::max<int64_t>(nv, 1));
  if (e == hipSuccess) e = b->vdir.ensure(sizeof(float4) * (size_t)std::max<int64_t>(b->n_direct, 1));
  if (e == hipSuccess) e = b->npart.ensure(sizeof(float4) * nq * (chunks.size() / 2));
  auto up = [&](DevBuf& d, const std::vector<int32_t>& h) {
    if (e == hipSuccess) e = d.ensure(sizeof(int32_t) * h.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d.p, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s);
  };
  up(b->nvis, nvis);
  up(b->nchunks, chunks);
  up(b->nchunk_first, chunk_first);
  up(b->dvis, dvis);
  up(b->dkey, dkey);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors go out of scope
  if (e != hipSuccess) return hip_fail(c, e, "gc_backward: visit indices");
  b->adj_nodes = n_nodes;
  b->adj_chunks = chunk_first[n_nodes];
  return GC_OK;
}

static hipError_t build_ranks(gc_batch b, hipStream_t s) {
  // union rank of every address-list entry: targets in task order, then direct entries
  std::vector<int32_t> ir((size_t)std::max<int64_t>(b->n_targets, 1)), jr((size_t)std::max<int64_t>(b->n_direct, 1));
  auto upos = [&](int32_t id) -> int32_t {
    return (int32_t)(std::lower_bound(b->hU.begin(), b->hU.end(), id) - b->hU.begin());
  };
  int64_t io = 0, jo = 0;
  for (const gc_task& tk : b->tasks) {
    const int32_t p0 = tk.i_count > 0 ? upos(tk.i_begin) : 0;
    for (int32_t k = 0; k < tk.i_count; ++k) ir[io++] = p0 + k;
    for (int32_t r = 0; r < tk.j_nranges; ++r) {
      const int32_t g0 = b->ranges[2 * (tk.j_first + r)], gn = b->ranges[2 * (tk.j_first + r) + 1];
      const int32_t q0 = gn > 0 ? upos(g0) : 0;
      for (int32_t k = 0; k < gn; ++k) jr[jo++] = q0 + k;
    }
  }
  hipError_t e = b->d_irank.ensure(sizeof(int32_t) * ir.size());
  if (e == hipSuccess) e = b->d_jrank.ensure(sizeof(int32_t) * jr.size());
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_irank.p, ir.data(), sizeof(int32_t) * ir.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_jrank.p, jr.data(), sizeof(int32_t) * jr.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors go out of scope
  if (e == hipSuccess) b->ranks_ready = true;
  return e;
}

static hipError_t ensure_reorg_buffers(gc_batch b, gc_pool p, int32_t mode, hipStream_t s) {
  const size_t u = (size_t)std::max<int32_t>(b->u, 1);
  const void* st0 = b->state.p;
  const void* fl0 = b->free_list.p;
  hipError_t e = b->uslot.ensure(sizeof(int32_t) * u);
  if (e == hipSuccess) e = b->missing.ensure(sizeof(int32_t) * u);
  if (e == hipSuccess) e = b->mslot.ensure(sizeof(int32_t) * u);
  if (e == hipSuccess) e = b->free_list.ensure(sizeof(uint64_t) * u);
  if (e == hipSuccess) e = b->state.ensure(sizeof(int32_t) * (size_t)reorg_state_ints(b->u, p->cap));
  if (e == hipSuccess) e = b->packed.ensure(sizeof(float4) * u);
  if (e == hipSuccess) e = b->queue.ensure(sizeof(int32_t) * 4);
  if (e == hipSuccess && lists_mode(mode)) {
    e = b->ilist.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(b->n_targets, 1));
    if (e == hipSuccess) e = b->jlist.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(b->n_direct, 1));
    if (e == hipSuccess && !b->ranks_ready) e = build_ranks(b, s);
  }
  if (e == hipSuccess && (b->state.p != st0 || b->free_list.p != fl0)) {
    e = launch_fill_i32(b->state.as<int32_t>(), 0, (int64_t)(b->state.bytes / 4), s);
    if (e == hipSuccess) e = launch_fill_i32(b->free_list.as<int32_t>(), 0, (int64_t)(b->free_list.bytes / 4), s);
  }
  return e;
}

// Clears the reorganisation state and the free-slot list (the staged set of the last call is forgotten).
static hipError_t clear_reorg_state(gc_batch b, hipStream_t s) {
  hipError_t e = launch_fill_i32(b->state.as<int32_t>(), 0, (int64_t)(b->state.bytes / 4), s);
  if (e == hipSuccess) e = launch_fill_i32(b->free_list.as<int32_t>(), 0, (int64_t)(b->free_list.bytes / 4), s);
  return e;
}

// Device part of a reorganisation (buffers already sized).  staged: the missing records, copied in
// from the host in missing order (host-staged calls; REDUNDANT then has its records in `packed`
// already).
static gc_status reorganize_async(gc_batch b, gc_pool p, int32_t mode, hipStream_t s, const float4* staged = nullptr) {
  gc_ctx c = b->ctx;
  if (mode == GC_REORG_REDUNDANT) {
    if (p->host_src)
      GC_HIP(c, launch_fill_i32(b->state.as<int32_t>() + GC_STATE_UNION, b->u, 2, s));  // |U| and #missing
    else
      GC_HIP(c, launch_gather_src(b->d_U.as<int32_t>(), b->u, p->src, b->packed.as<float4>(), b->state.as<int32_t>(),
                                  s));
  } else {
    ReorgArgs a{};
    a.U = b->d_U.as<int32_t>();
    a.u = b->u;
    a.src = p->src;
    a.staged = staged;
    a.pool = p->rec.as<float4>();
    a.slot_of = p->slot_of.as<int32_t>();
    a.occ = p->occ.as<uint32_t>();
    a.cap = p->cap;
    a.pack = mode == GC_REORG_PACK ? 1 : 0;
    a.packed = b->packed.as<float4>();
    a.uslot = b->uslot.as<int32_t>();
    a.missing = b->missing.as<int32_t>();
    a.mslot = b->mslot.as<int32_t>();
    a.free_list = b->free_list.as<uint64_t>();
    a.state = b->state.as<int32_t>();
    GC_HIP(c, launch_reorg(a, s));
    if (lists_mode(mode)) {
      GC_HIP(c, launch_lists(b->d_irank.as<int32_t>(), b->n_targets, b->d_jrank.as<int32_t>(), b->n_direct,
                             b->uslot.as<int32_t>(), b->ilist.as<int32_t>(), b->jlist.as<int32_t>(), s));
      if (mode == GC_REORG_SORTED)
        GC_HIP(c, launch_sort_lists(b->nt, b->d_joff.as<int32_t>(), b->jlist.as<int32_t>(), s));
    }
  }
  b->rec = (mode == GC_REORG_PACK || mode == GC_REORG_REDUNDANT) ? b->packed.as<float4>() : p->rec.as<float4>();
  b->staged_live = mode != GC_REORG_REDUNDANT;  // (REDUNDANT stages nothing into the pool)
  return GC_OK;
}

// Host-staged reorganisation (pool with a host source).  The host finds the missing records in its
// mirror of the chare table, packs them into the batch's pinned buffer and copies them to the
// device on `side` (REDUNDANT: every record of U, straight into the packed buffer); the kernel on
// `s` waits for the copy.  The copy waits only for earlier work on `s` that read this batch's
// staged or packed records, so it overlaps other batches' passes.
static gc_status reorganize_host(gc_batch b, gc_pool p, int32_t mode, int32_t check_capacity, hipStream_t s,
                                 hipStream_t side) {
  gc_ctx c = b->ctx;
  const bool redundant = mode == GC_REORG_REDUNDANT;
  gc_status hs = need_host_lists(b, s);
  if (hs != GC_OK) return hs;
  if (!redundant && !p->mirror_ok) GC_HIP(c, mirror_sync(p, s));
  // the missing ids, into the batch's own vector (kept across calls: its storage is reused, so the
  // call allocates no host memory once the batch has been reorganised)
  std::vector<int32_t>& miss = b->h_missing;
  miss.clear();
  if (!redundant) {
    // branch-free: about half of a round's ids are missing, in no predictable pattern
    miss.resize((size_t)b->u);
    const int32_t* so = p->m_slot_of.data();
    int32_t* out = miss.data();
    size_t n = 0;
    for (int32_t id : b->hU) {
      out[n] = id;
      n += so[id] < 0 ? 1 : 0;
    }
    miss.resize(n);
  }
  const int32_t* ids = redundant ? b->hU.data() : miss.data();
  const int64_t m = redundant ? b->u : (int64_t)miss.size();
  if (!redundant && check_capacity && m > p->m_nfree) {
    miss.clear();
    b->host_staged = false;
    b->mode = -1;
    return set_err(c, GC_E_FULL, "gc_reorganize: %lld records missing but only %lld pool slots free", (long long)m,
                   (long long)p->m_nfree);
  }
  b->mode = -1;
  hipError_t e = ensure_reorg_buffers(b, p, mode, s);
  // room for every union entry, so that the kernel's reads stay inside it whatever its own count
  if (e == hipSuccess && !redundant) e = b->staged.ensure(sizeof(float4) * (size_t)std::max<int32_t>(b->u, 1));
  if (e != hipSuccess) return set_err(c, GC_E_NOMEM, "gc_reorganize: %s", hipGetErrorString(e));
  GC_HIP(c, b->ev_copy.sync());  // the pinned buffer is free once its last copy has run
  if (b->pin.ensure(sizeof(float4) * (size_t)std::max<int64_t>(m, 1)) != hipSuccess)
    return set_err(c, GC_E_NOMEM, "gc_reorganize: pinned staging buffer");
  float4* pin = b->pin.as<float4>();
  for (int64_t k = 0; k < m; ++k) pin[k] = p->host_src[ids[k]];
  hipStream_t cs = side ? side : s;
  if (m > 0) {
    if (cs != s) GC_HIP(c, b->ev_use.wait(cs));
    GC_HIP(c, hipMemcpyAsync(redundant ? b->packed.p : b->staged.p, pin, sizeof(float4) * (size_t)m,
                             hipMemcpyHostToDevice, cs));
    GC_HIP(c, b->ev_copy.record(cs));
    if (cs != s) GC_HIP(c, b->ev_copy.wait(s));
  }
  gc_status st = reorganize_async(b, p, mode, s, redundant ? nullptr : b->staged.as<float4>());
  if (st != GC_OK) return st;
  GC_HIP(c, b->ev_use.record(s));
  b->h_mslot.resize((size_t)m);
  if (!redundant) mirror_assign(p, miss.data(), m, b->h_mslot.data());
  else miss.clear();
  b->host_staged = true;
  b->mode = mode;
  b->pool = p;
  return GC_OK;
}

extern "C" gc_status gc_reorganize(gc_batch b, gc_pool p, int32_t mode, int32_t check_capacity, void* stream,
                                   void* side_stream) {
  if (!b || !p) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (!b->committed) return set_err(c, GC_E_STATE, "gc_reorganize: batch not committed");
  if (p->n_ids != b->n_ids) return set_err(c, GC_E_INVAL, "gc_reorganize: pool and batch id spaces differ");
  if (mode < GC_REORG_REDUNDANT || mode > GC_REORG_NONE) return set_err(c, GC_E_INVAL, "gc_reorganize: bad mode %d", mode);
  if (!p->src && !p->host_src) return set_err(c, GC_E_STATE, "gc_reorganize: pool has no source");
  if (mode == GC_REORG_SORTED && b->max_direct > kSortMax)
    return set_err(c, GC_E_UNSUPPORTED, "gc_reorganize: SORTED supports at most %d direct entries per task (got %d)",
                   kSortMax, b->max_direct);
  if (p->host_src) {
    if (mode == GC_REORG_NONE) return set_err(c, GC_E_INVAL, "gc_reorganize: NONE needs a device-resident source");
    return reorganize_host(b, p, mode, check_capacity, S(stream), S(side_stream));
  }
  b->host_staged = false;
  p->mirror_ok = false;
  if (mode == GC_REORG_NONE) {
    if (!p->src_device) return set_err(c, GC_E_INVAL, "gc_reorganize: NONE needs a device-resident source");
    b->mode = mode;
    b->pool = p;
    b->rec = p->src;
    return GC_OK;
  }
  hipStream_t s = S(stream);
  if (lists_mode(mode)) {  // the address lists' union ranks are built on the host
    gc_status hs = need_host_lists(b, s);
    if (hs != GC_OK) return hs;
  }
  b->mode = -1;
  hipError_t e = ensure_reorg_buffers(b, p, mode, s);
  if (e != hipSuccess) return set_err(c, GC_E_NOMEM, "gc_reorganize: %s", hipGetErrorString(e));
  if (check_capacity && mode != GC_REORG_REDUNDANT) {
    // count first (no side effects), so that a full pool is reported with the pool unchanged
    int32_t* st = b->state.as<int32_t>();
    GC_HIP(c, launch_fill_i32(st + GC_STATE_CHECK, 0, 2, s));
    GC_HIP(c, launch_count(b->d_U.as<int32_t>(), b->u, p->slot_of.as<int32_t>(), p->occ.as<uint32_t>(), p->cap,
                           st + GC_STATE_CHECK, s));
    int32_t h[8];
    GC_HIP(c, hipMemcpyAsync(h, st, sizeof h, hipMemcpyDeviceToHost, s));
    GC_HIP(c, hipStreamSynchronize(s));
    if (h[GC_STATE_ERR]) return set_err(c, GC_E_HIP, "gc_reorganize: an earlier reorganisation hit a wait bound");
    if (h[GC_STATE_CHECK] > h[GC_STATE_CHECK + 1])
      return set_err(c, GC_E_FULL, "gc_reorganize: %d records missing but only %d pool slots free", h[GC_STATE_CHECK],
                     h[GC_STATE_CHECK + 1]);
  }
  gc_status st = reorganize_async(b, p, mode, s);
  if (st != GC_OK) return st;
  b->mode = mode;
  b->pool = p;
  return GC_OK;
}

extern "C" gc_status gc_pool_evict(gc_pool pool, const int32_t* ids_dev, int32_t n, void* stream) {
  if (!pool) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (n < 0 || (n > 0 && !ids_dev)) return set_err(pool->ctx, GC_E_INVAL, "gc_pool_evict: bad arrays");
  if (pool->host_src && pool->mirror_ok && n > 0) {
    std::vector<int32_t> ids;
    GC_HIP(pool->ctx, read_ids(ids_dev, n, ids, S(stream)));
    for (int32_t id : ids)
      if (id >= 0 && id < pool->n_ids) mirror_free_id(pool, id);
  }
  GC_HIP(pool->ctx, launch_evict(ids_dev, nullptr, n, pool->slot_of.as<int32_t>(), pool->n_ids,
                                 pool->occ.as<uint32_t>(), S(stream)));
  return GC_OK;
}

static gc_status evict_staged_async(gc_pool pool, gc_batch b, hipStream_t s) {
  if (b->mode != GC_REORG_PACK && b->mode != GC_REORG_INDIRECT && b->mode != GC_REORG_SORTED) return GC_OK;
  if (pool->host_src && pool->mirror_ok) {
    if (b->host_staged) {
      for (size_t k = 0; k < b->h_missing.size(); ++k)
        if (b->h_mslot[k] >= 0) mirror_free_id(pool, b->h_missing[k]);
    } else {
      pool->mirror_ok = false;
    }
  }
  GC_HIP(pool->ctx, launch_evict(b->missing.as<int32_t>(), b->state.as<int32_t>() + GC_STATE_MISSING,
                                 std::max<int32_t>(b->u, 1), pool->slot_of.as<int32_t>(), pool->n_ids,
                                 pool->occ.as<uint32_t>(), s));
  return GC_OK;
}

extern "C" gc_status gc_pool_evict_staged(gc_pool pool, gc_batch b, void* stream) {
  if (!pool || !b) return GC_E_INVAL;
  GC_ENTER(pool->ctx);
  if (b->mode < 0 || !b->pool) return GC_OK;  // nothing staged yet
  if (b->pool != pool) return set_err(pool->ctx, GC_E_STATE, "gc_pool_evict_staged: batch last reorganised against another pool");
  gc_status st = evict_staged_async(pool, b, S(stream));
  if (st == GC_OK) b->staged_live = false;
  return st;
}

extern "C" gc_status gc_batch_maps(gc_batch b, int64_t* counts, int32_t* U, int32_t* pos, int32_t* missing,
                                   int32_t* new_slot, int32_t* pranges, int32_t* pi_begin, int32_t* ilist,
                                   int32_t* jlist, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (b->mode < 0 || b->mode == GC_REORG_NONE) return set_err(c, GC_E_STATE, "gc_batch_maps: no reorganisation");
  hipStream_t s = S(stream);
  gc_status hs = need_host_lists(b, s);
  if (hs != GC_OK) return hs;
  int32_t h[8];
  GC_HIP(c, hipMemcpyAsync(h, b->state.p, sizeof h, hipMemcpyDeviceToHost, s));
  GC_HIP(c, hipStreamSynchronize(s));
  if (h[GC_STATE_ERR]) return set_err(c, GC_E_HIP, "gc_batch_maps: a reorganisation wait hit its bound");
  if (b->mode != GC_REORG_REDUNDANT && h[GC_STATE_MISSING] > h[GC_STATE_FREE])
    return set_err(c, GC_E_FULL, "gc_batch_maps: the last reorganisation overflowed the pool");
  const int32_t nu = b->u, nm = (b->mode == GC_REORG_REDUNDANT) ? b->u : h[GC_STATE_MISSING];
  if (counts) {
    counts[0] = nu;
    counts[1] = nm;
  }
  auto dn = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || !bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
  };
  if (b->mode == GC_REORG_REDUNDANT) {
    if (missing && nu) std::memcpy(missing, b->hU.data(), sizeof(int32_t) * (size_t)nu);
  } else {
    GC_HIP(c, dn(missing, b->missing.p, sizeof(int32_t) * (size_t)nm));
    GC_HIP(c, dn(new_slot, b->mslot.p, sizeof(int32_t) * (size_t)nm));
  }
  if (b->mode == GC_REORG_PACK || b->mode == GC_REORG_REDUNDANT) {
    GC_HIP(c, dn(pranges, b->pranges.p, sizeof(int32_t) * 2 * (size_t)b->nr));
    GC_HIP(c, dn(pi_begin, b->pibeg.p, sizeof(int32_t) * (size_t)b->nt));
  } else {
    GC_HIP(c, dn(ilist, b->ilist.p, sizeof(int32_t) * (size_t)b->n_targets));
    GC_HIP(c, dn(jlist, b->jlist.p, sizeof(int32_t) * (size_t)b->n_direct));
  }
  GC_HIP(c, hipStreamSynchronize(s));
  if (U && nu) std::memcpy(U, b->hU.data(), sizeof(int32_t) * (size_t)nu);
  if (pos) {
    for (int32_t i = 0; i < b->n_ids; ++i) pos[i] = -1;
    for (int32_t k = 0; k < nu; ++k) pos[b->hU[k]] = k;
  }
  return GC_OK;
}

// ===================================================================== combined launch

static gc_status check_prm(gc_batch b, const gc_force_params* prm, int* tile, int* wpb) {
  gc_ctx c = b->ctx;
  if (!prm) return set_err(c, GC_E_INVAL, "NULL force parameters");
  if (b->kind == GC_KIND_GRAV && prm->kind != GC_FORCE_GRAV_MONO && prm->kind != GC_FORCE_GRAV_QUAD)
    return set_err(c, GC_E_INVAL, "gravity batch needs GC_FORCE_GRAV_MONO or GC_FORCE_GRAV_QUAD");
  if (b->kind == GC_KIND_LJ && prm->kind != GC_FORCE_LJ) return set_err(c, GC_E_INVAL, "LJ batch needs GC_FORCE_LJ");
  *tile = prm->tile ? prm->tile : 256;
  *wpb = prm->waves_per_block ? prm->waves_per_block : 4;
  if (*tile < 64 || *tile > kMaxTile || *tile % 64) return set_err(c, GC_E_INVAL, "tile must be a multiple of 64 in [64, %d]", kMaxTile);
  if (*wpb < 1 || *wpb > 8) return set_err(c, GC_E_INVAL, "waves_per_block must be in [1, 8]");
  if (b->kind == GC_KIND_GRAV && !(prm->soft_eps > 0.f)) return set_err(c, GC_E_INVAL, "soft_eps must be > 0");
  if (b->kind == GC_KIND_LJ) {
    if (prm->n_types < 1 || prm->n_types > 8 || !prm->eps_t || !prm->sig_t || !prm->mass_t)
      return set_err(c, GC_E_INVAL, "LJ needs 1..8 types and device eps_t, sig_t, mass_t");
    if (!(prm->r_cut > 0.f)) return set_err(c, GC_E_INVAL, "r_cut must be > 0");
    *wpb = 4;
  }
  if (prm->schedule < GC_SCHED_TASKS || prm->schedule > GC_SCHED_ROUNDS)
    return set_err(c, GC_E_INVAL, "schedule must be GC_SCHED_TASKS, GC_SCHED_QUEUE, GC_SCHED_STEP or GC_SCHED_ROUNDS");
  if (prm->targets_per_lane < 0 || prm->targets_per_lane > 3)
    return set_err(c, GC_E_INVAL, "targets_per_lane must be 0, 1, 2 or 3");
  if (b->kind == GC_KIND_GRAV && b->max_node >= prm->n_nodes)
    return set_err(c, GC_E_INVAL, "node index %d is not below n_nodes %d of the node table", b->max_node, prm->n_nodes);
  // the force code forms node offsets with 24-bit multiplies and splits a task's direct records in
  // 32-bit arithmetic
  if (b->kind == GC_KIND_GRAV && prm->n_nodes > (1 << 24))
    return set_err(c, GC_E_UNSUPPORTED, "node tables of more than 2^24 nodes are not supported (got %d)", prm->n_nodes);
  if (b->kind == GC_KIND_GRAV && b->max_direct >= (1 << 28))
    return set_err(c, GC_E_UNSUPPORTED, "a task with 2^28 or more direct records is not supported");
  if (prm->want_potential != 0 && prm->want_potential != 1) return set_err(c, GC_E_INVAL, "want_potential must be 0 or 1");
  if (prm->deterministic != 0 && prm->deterministic != 1) return set_err(c, GC_E_INVAL, "deterministic must be 0 or 1");
  if (prm->aggregation < 0) return set_err(c, GC_E_INVAL, "aggregation must be >= 0");
  if (prm->aggregation > 0 && b->kind != GC_KIND_GRAV)
    return set_err(c, GC_E_UNSUPPORTED, "aggregation counts are for gravity batches (Lennard-Jones runs one launch)");
  return GC_OK;
}

static gc_status launch_combined_async(gc_batch b, const gc_force_params* prm, const float* nodes_dev, float* acc_dev,
                                       hipStream_t s) {
  gc_ctx c = b->ctx;
  int tile, wpb;
  gc_status st = check_prm(b, prm, &tile, &wpb);
  if (st != GC_OK) return st;
  if (prm->schedule == GC_SCHED_STEP || prm->schedule == GC_SCHED_ROUNDS)
    return set_err(c, GC_E_UNSUPPORTED, "the whole-step and rounds schedules run through gc_graph_capture only");
  if (b->mode < 0 || !b->pool) return set_err(c, GC_E_STATE, "gc_launch_combined: batch not reorganised");
  if (!acc_dev) return set_err(c, GC_E_INVAL, "gc_launch_combined: NULL acc");
  if (prm->want_potential && b->kind == GC_KIND_LJ)
    return set_err(c, GC_E_UNSUPPORTED, "gc_launch_combined: the potential is written for gravity only");
  if (prm->want_potential && (b->mode == GC_REORG_INDIRECT || b->mode == GC_REORG_SORTED))
    return set_err(c, GC_E_UNSUPPORTED, "gc_launch_combined: the potential needs PACK, REDUNDANT or NONE");
  if (prm->deterministic && b->kind == GC_KIND_LJ && !b->lj_gather)
    return set_err(c, GC_E_UNSUPPORTED,
                   "gc_launch_combined: this Lennard-Jones batch (target ranges that partially overlap) sums with "
                   "atomics; no deterministic form");
  const int32_t T = b->nt;
  const bool packed = (b->mode == GC_REORG_PACK || b->mode == GC_REORG_REDUNDANT);
  const bool lists = (b->mode == GC_REORG_INDIRECT || b->mode == GC_REORG_SORTED);
  const bool persistent = prm->schedule == 1;
  if (b->queue.ensure(16) != hipSuccess) return set_err(c, GC_E_NOMEM, "queue");
  if (persistent) GC_HIP(c, launch_fill_i32(b->queue.as<int32_t>(), 0, 1, s));
  if (b->kind == GC_KIND_GRAV) {
    if (!nodes_dev && b->nn) return set_err(c, GC_E_INVAL, "gc_launch_combined: NULL nodes with node refs");
    GravArgs a{};
    a.tasks = b->d_tasks.as<gc_task>();
    a.n_tasks = T;
    a.ranges = packed ? b->pranges.as<int2>() : b->d_ranges.as<int2>();
    a.ibeg = packed ? b->pibeg.as<int32_t>() : nullptr;
    a.ioff = b->d_ioff.as<int32_t>();
    a.joff = b->d_joff.as<int32_t>();
    a.ilist = b->ilist.as<int32_t>();
    a.jlist = b->jlist.as<int32_t>();
    a.node_idx = b->d_nodes.as<int32_t>();
    a.nodes = reinterpret_cast<const float4*>(nodes_dev);
    a.n_nodes = prm->n_nodes;
    a.rec = b->rec;
    a.acc = reinterpret_cast<float4*>(acc_dev);
    a.G = prm->G;
    a.eps2 = prm->soft_eps * prm->soft_eps;
    a.tile = tile;
    a.queue = b->queue.as<int32_t>();
    a.order = b->d_order.as<int32_t>();
    int order = prm->kind == GC_FORCE_GRAV_QUAD ? 2 : 1;
    const int tpl = prm->targets_per_lane == 0 ? 1 : prm->targets_per_lane;
    int grid = prm->grid_blocks;
    if (persistent && grid <= 0) {
      int per = 0;
      GC_HIP(c, grav_occupancy(order, lists, true, tpl, tile, wpb, &per));
      grid = std::max(1, per) * c->n_cu;
    }
    // aggregation: consecutive launches over slices of the launch order (each slice's queue counter
    // is its own word, so the persistent form needs no reset between them)
    const int32_t agg = prm->aggregation > 0 && prm->aggregation < T ? prm->aggregation : T;
    const int32_t n_launch = T > 0 ? (T + agg - 1) / agg : 0;
    if (persistent && n_launch > 1) {
      if (b->queue.ensure(sizeof(int32_t) * (size_t)(n_launch + 4)) != hipSuccess)
        return set_err(c, GC_E_NOMEM, "queue");
      GC_HIP(c, launch_fill_i32(b->queue.as<int32_t>(), 0, n_launch, s));
    }
    if (prm->want_potential) {
      for (int32_t q = 0; q < n_launch; ++q) {
        GravArgs aq = a;
        aq.order = b->d_order.as<int32_t>() + (int64_t)q * agg;
        aq.n_tasks = std::min<int32_t>(agg, T - q * agg);
        GC_HIP(c, launch_grav_potential(order, aq, wpb, s));
      }
      return GC_OK;
    }
    for (int32_t q = 0; q < n_launch; ++q) {
      GravArgs aq = a;
      aq.order = b->d_order.as<int32_t>() + (int64_t)q * agg;
      aq.n_tasks = std::min<int32_t>(agg, T - q * agg);
      aq.queue = b->queue.as<int32_t>() + (n_launch > 1 ? q : 0);
      GC_HIP(c, launch_grav(order, lists, persistent, tpl, aq, wpb, grid, s));
    }
  } else {
    if (lists) return set_err(c, GC_E_UNSUPPORTED, "Lennard-Jones supports PACK, REDUNDANT and NONE");
    if (!b->pool->src_device) return set_err(c, GC_E_INVAL, "Lennard-Jones needs a device-resident source");
    if (!b->lj_gather || !b->lj_cover) GC_HIP(c, launch_fill_f32(acc_dev, 0.f, 4 * (int64_t)b->n_ids, s));
    LJArgs a{};
    a.tasks = b->d_tasks.as<gc_task>();
    a.n_tasks = T;
    a.ranges = packed ? b->pranges.as<int2>() : b->d_ranges.as<int2>();
    a.ranges_id = b->d_ranges.as<int2>();
    a.ibeg = packed ? b->pibeg.as<int32_t>() : nullptr;
    a.rec = b->rec;
    a.acc = reinterpret_cast<float4*>(acc_dev);
    a.eps_t = prm->eps_t;
    a.sig_t = prm->sig_t;
    a.n_types = prm->n_types;
    a.rc2 = prm->r_cut * prm->r_cut;
    a.queue = b->queue.as<int32_t>();
    a.order = b->d_order.as<int32_t>();
    a.runs = b->d_runs.as<int32_t>();
    a.n_runs = b->n_runs;
    a.tgt = b->d_ljtgt.as<int4>();
    a.ent = b->d_ljent.as<int32_t>();
    a.n_tgt = b->n_ljtgt;
    a.mass_t = prm->mass_t;
    if (b->lj_gather) {
      GC_HIP(c, launch_lj_gather(persistent, a, prm->grid_blocks > 0 ? prm->grid_blocks : 5 * c->n_cu, s));
    } else {
      int grid = prm->grid_blocks > 0 ? prm->grid_blocks : 8 * c->n_cu;
      GC_HIP(c, launch_lj(persistent, a, 4, grid, s));
      GC_HIP(c, launch_lj_finish(reinterpret_cast<float4*>(acc_dev), prm->mass_t, b->pool->src, b->n_ids, s));
    }
  }
  return GC_OK;
}

extern "C" gc_status gc_launch_combined(gc_batch b, const gc_force_params* prm, const float* nodes_dev, float* acc_dev,
                                        void* stream) {
  if (!b) return GC_E_INVAL;
  GC_ENTER(b->ctx);
  gc_status st = launch_combined_async(b, prm, nodes_dev, acc_dev, S(stream));
  // a host-staged batch's next copy waits for this pass's reads of its records
  if (st == GC_OK && b->host_staged) GC_HIP(b->ctx, b->ev_use.record(S(stream)));
  return st;
}

extern "C" gc_status gc_lj_count_pairs(gc_batch b, float r_cut, int64_t* pairs, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (!pairs) return set_err(c, GC_E_INVAL, "gc_lj_count_pairs: NULL output");
  if (b->kind != GC_KIND_LJ) return set_err(c, GC_E_INVAL, "gc_lj_count_pairs: Lennard-Jones batches only");
  if (!(r_cut > 0.f)) return set_err(c, GC_E_INVAL, "gc_lj_count_pairs: r_cut must be > 0");
  if (!b->committed || b->mode < 0 || !b->pool) return set_err(c, GC_E_STATE, "gc_lj_count_pairs: batch not reorganised");
  if (!b->pool->src_device) return set_err(c, GC_E_INVAL, "gc_lj_count_pairs: needs a device-resident source");
  hipStream_t s = S(stream);
  if (b->queue.ensure(16) != hipSuccess) return set_err(c, GC_E_NOMEM, "gc_lj_count_pairs: counter");
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(b->queue.as<int32_t>() + 2);
  GC_HIP(c, launch_fill_i32(b->queue.as<int32_t>() + 2, 0, 2, s));
  GC_HIP(c, launch_lj_count(b->d_tasks.as<gc_task>(), b->nt, b->d_ranges.as<int2>(), b->pool->src, r_cut * r_cut, cnt,
                            s));
  unsigned long long h = 0;
  GC_HIP(c, hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  GC_HIP(c, hipStreamSynchronize(s));
  *pairs = (int64_t)h;
  return GC_OK;
}

extern "C" gc_status gc_occupancy(gc_ctx ctx, const gc_force_params* prm, int32_t* blocks_per_cu, int32_t* n_cu) {
  GC_ENTER(ctx);
  if (!prm || !blocks_per_cu) return set_err(ctx, GC_E_INVAL, "gc_occupancy: NULL argument");
  int tile = prm->tile ? prm->tile : 256, wpb = prm->waves_per_block ? prm->waves_per_block : 4, per = 0;
  const int order = prm->kind == GC_FORCE_GRAV_QUAD ? 2 : 1;
  const int tpl = prm->targets_per_lane == 0 ? 1 : prm->targets_per_lane;
  if (prm->schedule == GC_SCHED_STEP)
    GC_HIP(ctx, step_occupancy(order, tpl, tile, &per));
  else
    GC_HIP(ctx, grav_occupancy(order, false, prm->schedule == GC_SCHED_QUEUE, tpl, tile, wpb, &per));
  *blocks_per_cu = per;
  if (n_cu) *n_cu = ctx->n_cu;
  return GC_OK;
}

// ===================================================================== Ewald correction

extern "C" gc_status gc_launch_ewald(gc_batch b, const gc_ewald_params* prm, float* acc_dev, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (!prm || !acc_dev) return set_err(c, GC_E_INVAL, "gc_launch_ewald: NULL argument");
  if (b->kind != GC_KIND_GRAV) return set_err(c, GC_E_INVAL, "gc_launch_ewald: gravity batches only");
  bool s_finite = true;
  for (int k = 0; k < 6; ++k) s_finite = s_finite && std::isfinite(prm->S[k]);
  if (!(prm->L > 0.f) || !(prm->alpha >= 0.f) || prm->nrep < 0 || prm->nrep > 4 || prm->hmax2 < 0 ||
      prm->hmax2 > kEwaldMaxHmax2 || !s_finite)
    return set_err(c, GC_E_INVAL,
                   "gc_launch_ewald: need L > 0, alpha >= 0, 0 <= nrep <= 4, 0 <= hmax2 <= %d, finite S",
                   kEwaldMaxHmax2);
  if (b->mode < 0 || !b->pool) return set_err(c, GC_E_STATE, "gc_launch_ewald: batch not reorganised");
  if (lists_mode(b->mode)) return set_err(c, GC_E_UNSUPPORTED, "gc_launch_ewald: PACK, REDUNDANT or NONE");
  const bool packed = (b->mode == GC_REORG_PACK || b->mode == GC_REORG_REDUNDANT);
  EwaldArgs a{};
  a.tasks = b->d_tasks.as<gc_task>();
  a.n_tasks = b->nt;
  a.ioff = b->d_ioff.as<int32_t>();
  a.n_targets = b->n_targets;
  a.ibeg = packed ? b->pibeg.as<int32_t>() : nullptr;
  a.rec = b->rec;
  a.acc = reinterpret_cast<float4*>(acc_dev);
  a.L = prm->L;
  a.inv_L = 1.f / prm->L;
  a.alpha = prm->alpha > 0.f ? prm->alpha : 2.f / prm->L;
  a.GM = prm->G * prm->M;
  for (int d = 0; d < 3; ++d) a.c[d] = prm->com[d];
  a.nrep = prm->nrep;
  a.hmax2 = prm->hmax2;
  a.hmax = 0;
  while ((a.hmax + 1) * (a.hmax + 1) <= a.hmax2) ++a.hmax;
  a.kcoef = -2.f * a.GM / (prm->L * prm->L);
  const double aL = (double)a.alpha * prm->L;
  a.kdecay = (float)(M_PI * M_PI / (aL * aL));
  a.quad = false;
  for (int k = 0; k < 6; ++k) {
    a.GS[k] = prm->G * prm->S[k];
    a.quad = a.quad || prm->S[k] != 0.f;
  }
  const double L2 = (double)prm->L * prm->L;
  a.qcoef = (float)(4.0 * M_PI * M_PI / (L2 * L2));
  GC_HIP(c, launch_ewald(a, S(stream)));
  if (b->host_staged) GC_HIP(c, b->ev_use.record(S(stream)));
  return GC_OK;
}

// ===================================================================== combining policy (Sec. 3.1)

struct gc_combiner_ {
  int32_t max_size = 1;
  int64_t waiting = 0;
  bool any = false;        // an arrival has been seen
  double t_last = 0.0;     // time of the last arrival
  double t_now = 0.0;      // latest time given (arrive or poll)
  double max_interval = 0.0;
  int64_t n_full = 0, n_idle = 0;
};

extern "C" gc_status gc_combiner_create(int32_t max_size, gc_combiner* out) {
  if (!out || max_size < 1) return GC_E_INVAL;
  gc_combiner c = new (std::nothrow) gc_combiner_();
  if (!c) return GC_E_NOMEM;
  c->max_size = max_size;
  *out = c;
  return GC_OK;
}

extern "C" gc_status gc_combiner_destroy(gc_combiner c) {
  if (!c) return GC_E_INVAL;
  delete c;
  return GC_OK;
}

extern "C" gc_status gc_combiner_arrive(gc_combiner c, double t, int64_t n) {
  if (!c || n < 1 || !(t >= c->t_now)) return GC_E_INVAL;
  if (c->any) c->max_interval = std::max(c->max_interval, t - c->t_last);
  c->any = true;
  c->t_last = t;
  c->t_now = t;
  c->waiting += n;
  return GC_OK;
}

extern "C" gc_status gc_combiner_poll(gc_combiner c, double t, int64_t* take, int32_t* reason) {
  if (!c || !take || !(t >= c->t_now)) return GC_E_INVAL;
  c->t_now = t;
  int64_t k = 0;
  int32_t why = 0;
  if (c->waiting >= c->max_size) {
    k = c->max_size;
    why = 1;
    ++c->n_full;
  } else if (c->waiting > 0 && t - c->t_last > 2.0 * c->max_interval) {
    k = c->waiting;
    why = 2;
    ++c->n_idle;
  }
  c->waiting -= k;
  *take = k;
  if (reason) *reason = why;
  return GC_OK;
}

extern "C" gc_status gc_combiner_state(gc_combiner c, int64_t* waiting, double* max_interval, int64_t* n_full,
                                       int64_t* n_idle) {
  if (!c) return GC_E_INVAL;
  if (waiting) *waiting = c->waiting;
  if (max_interval) *max_interval = c->max_interval;
  if (n_full) *n_full = c->n_full;
  if (n_idle) *n_idle = c->n_idle;
  return GC_OK;
}

// ===================================================================== backward (adjoint)

extern "C" gc_status gc_backward(gc_batch b, const gc_force_params* prm, const float* nodes_dev,
                                 const int32_t* node_range_dev, int32_t n_nodes, const float* cot_dev, float* gpos_dev,
                                 float* gmass_dev, float* gparam_dev, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  int tile, wpb;
  gc_status st = check_prm(b, prm, &tile, &wpb);
  if (st != GC_OK) return st;
  if (b->mode < 0 || !b->pool) return set_err(c, GC_E_STATE, "gc_backward: batch not reorganised");
  if (prm->deterministic && (b->kind == GC_KIND_GRAV || !b->lj_gather))
    return set_err(c, GC_E_UNSUPPORTED, "gc_backward: this adjoint adds target gradients with atomics; no "
                                        "deterministic form");
  if (b->mode == GC_REORG_INDIRECT || b->mode == GC_REORG_SORTED)
    return set_err(c, GC_E_UNSUPPORTED, "gc_backward supports PACK, REDUNDANT and NONE reorganisations");
  if (!b->pool->src_device) return set_err(c, GC_E_INVAL, "gc_backward needs a device-resident source");
  if (!cot_dev || !gpos_dev || !gmass_dev) return set_err(c, GC_E_INVAL, "gc_backward: NULL cotangent or gradient");
  hipStream_t s = S(stream);
  const int32_t T = b->nt;
  const bool packed = (b->mode == GC_REORG_PACK || b->mode == GC_REORG_REDUNDANT);
  if (b->kind == GC_KIND_GRAV) {
    const int order = prm->kind == GC_FORCE_GRAV_QUAD ? 2 : 1;
    if (b->nn && (!nodes_dev || !node_range_dev || n_nodes <= 0))
      return set_err(c, GC_E_INVAL, "gc_backward: node table and node ranges needed");
    if (b->adj_nodes != std::max<int32_t>(n_nodes, 0)) {
      gc_status bst = build_adj_index(b, std::max<int32_t>(n_nodes, 0), s);
      if (bst != GC_OK) return bst;
    }
    GravAdjArgs a{};
    a.f.tasks = b->d_tasks.as<gc_task>();
    a.f.n_tasks = T;
    a.f.ranges = packed ? b->pranges.as<int2>() : b->d_ranges.as<int2>();
    a.f.ibeg = packed ? b->pibeg.as<int32_t>() : nullptr;
    a.f.node_idx = b->d_nodes.as<int32_t>();
    a.f.nodes = reinterpret_cast<const float4*>(nodes_dev);
    a.f.n_nodes = prm->n_nodes;
    a.f.rec = b->rec;
    a.f.G = prm->G;
    a.f.eps2 = prm->soft_eps * prm->soft_eps;
    a.cot = reinterpret_cast<const float4*>(cot_dev);
    a.gpos = reinterpret_cast<float4*>(gpos_dev);
    a.gmass = gmass_dev;
    a.src_id = packed ? b->d_U.as<int32_t>() : nullptr;
    a.joff = b->d_joff.as<int32_t>();
    a.vnode = b->vnode.as<float4>();
    a.vdir = b->vdir.as<float4>();
    // waves per task, measured on Plummer 262,144 (quadrupole) and uniform 4,096 (monopole)
    GC_HIP(c, launch_grav_adjoint(packed, order, a, order == 2 ? 2 : 4, s));
    if (b->n_direct > 0)
      GC_HIP(c, launch_direct_sums(a.vdir, b->dvis.as<int32_t>(), b->dkey.as<int32_t>(), (int32_t)b->n_direct,
                                   a.gpos, gmass_dev, s));
    if (b->nn) {
      GC_HIP(c, launch_visit_sums(order, a.vnode, b->nvis.as<int32_t>(), b->nchunks.as<int2>(), b->adj_chunks,
                                  b->npart.as<float4>(), s));
      GC_HIP(c, launch_node_chain(order, node_range_dev, n_nodes, reinterpret_cast<const float4*>(nodes_dev),
                                  b->npart.as<float4>(), b->nchunk_first.as<int32_t>(), b->pool->src, b->n_ids,
                                  a.gpos, gmass_dev, b->stat.as<int32_t>(), s));
    }
    return GC_OK;
  }
  if (!gparam_dev) return set_err(c, GC_E_INVAL, "gc_backward: Lennard-Jones needs gparam");
  if (b->force.ensure(sizeof(float4) * (size_t)b->n_ids) != hipSuccess)
    return set_err(c, GC_E_NOMEM, "gc_backward: force buffer");
  if (!b->lj_gather || !b->lj_cover) GC_HIP(c, launch_fill_f32(b->force.as<float>(), 0.f, 4 * (int64_t)b->n_ids, s));
  LJAdjArgs a{};
  a.f.tasks = b->d_tasks.as<gc_task>();
  a.f.n_tasks = T;
  a.f.ranges = packed ? b->pranges.as<int2>() : b->d_ranges.as<int2>();
  a.f.ranges_id = b->d_ranges.as<int2>();
  a.f.ibeg = packed ? b->pibeg.as<int32_t>() : nullptr;
  a.f.rec = b->rec;
  a.f.eps_t = prm->eps_t;
  a.f.sig_t = prm->sig_t;
  a.f.n_types = prm->n_types;
  a.f.rc2 = prm->r_cut * prm->r_cut;
  a.f.runs = b->d_runs.as<int32_t>();
  a.f.n_runs = b->n_runs;
  a.cot = reinterpret_cast<const float4*>(cot_dev);
  a.mass_t = prm->mass_t;
  a.gpos = reinterpret_cast<float4*>(gpos_dev);
  a.gparam = gparam_dev;
  a.force = b->force.as<float4>();
  a.f.tgt = b->d_ljtgt.as<int4>();
  a.f.ent = b->d_ljent.as<int32_t>();
  a.f.n_tgt = b->n_ljtgt;
  {
    const size_t rows = (size_t)std::max(1, lj_adjoint_blocks(a.f, b->lj_gather));
    if (b->ppart.ensure(sizeof(float) * rows * 2 * prm->n_types * prm->n_types) != hipSuccess)
      return set_err(c, GC_E_NOMEM, "gc_backward: parameter partials");
    a.ppart = b->ppart.as<float>();
  }
  if (b->lj_gather) GC_HIP(c, launch_lj_adjoint_gather(a, s));
  else GC_HIP(c, launch_lj_adjoint(a, 4, s));
  GC_HIP(c, launch_lj_mass_grad(a.cot, a.force, prm->mass_t, b->pool->src, gmass_dev, b->n_ids, s));
  return GC_OK;
}

// ===================================================================== graphs

// The whole-step schedule: every step's reorganisation and combined pass in one persistent launch
// (k_step).  Gravity, PACK, one pool, fixture NONE or EVICT_STAGED, distinct batches.
// combined_pass (GC_SCHED_ROUNDS): the persistent launch runs only the reorganisation items, and one
// combined launch after it runs every task of every round.
static gc_status capture_step(gc_ctx ctx, int32_t R, gc_batch* batches, gc_pool* pools, const int32_t* modes,
                              const gc_force_params* prm, const float* nodes_dev, float* acc_dev, int32_t fixture,
                              hipStream_t s, gc_graph gr, bool combined_pass) {
  gc_pool p = pools[0];
  if (fixture != GC_FIXTURE_NONE && fixture != GC_FIXTURE_EVICT_STAGED)
    return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: fixture must be NONE or EVICT_STAGED");
  if (prm->want_potential)
    return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: no potential output (use the per-round passes)");
  int tile = 256, wpb = 4;
  for (int32_t k = 0; k < R; ++k) {
    gc_batch b = batches[k];
    if (pools[k] != p) return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: one pool for all steps");
    if (modes[k] != GC_REORG_PACK) return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: PACK steps only");
    if (b->kind != GC_KIND_GRAV) return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: gravity batches only");
    for (int32_t q = 0; q < k; ++q)
      if (batches[q] == b) return set_err(ctx, GC_E_UNSUPPORTED, "whole-step schedule: distinct batches only");
    gc_status st = check_prm(b, prm, &tile, &wpb);
    if (st != GC_OK) return st;
    if (b->nn && !nodes_dev) return set_err(ctx, GC_E_INVAL, "whole-step schedule: NULL nodes");
  }
  if (!acc_dev) return set_err(ctx, GC_E_INVAL, "whole-step schedule: NULL acc");
  const int order = prm->kind == GC_FORCE_GRAV_QUAD ? 2 : 1;
  std::vector<StepRound> rounds((size_t)R);
  std::vector<StepItem> items;
  auto seg = [&](int32_t type, int32_t round, int32_t count) {
    for (int32_t i = 0; i < count; ++i) {
      StepItem it{};
      it.kind = type | round << 2;
      it.idx = i;
      if (type == kItemForce) {
        // the round's tasks in its launch order, each with its first packed target
        const gc_batch fb = batches[round];
        const int32_t t = fb->h_order[(size_t)i];
        const gc_task& tk = fb->tasks[(size_t)t];
        it.idx = fb->h_pibeg[(size_t)t];
        it.i_begin = tk.i_begin;
        it.i_count = tk.i_count;
        it.j_first = tk.j_first;
        it.j_nranges = tk.j_nranges;
        it.n_first = tk.n_first;
        it.n_count = tk.n_count;
      }
      items.push_back(it);
    }
  };
  for (int32_t k = 0; k < R; ++k) {
    gc_batch b = batches[k];
    StepRound& sr = rounds[k];
    GravArgs& g = sr.grav;
    g = GravArgs{};
    g.tasks = b->d_tasks.as<gc_task>();
    g.n_tasks = (int32_t)b->tasks.size();
    g.ranges = b->pranges.as<int2>();
    g.ibeg = b->pibeg.as<int32_t>();
    g.ioff = b->d_ioff.as<int32_t>();
    g.joff = b->d_joff.as<int32_t>();
    g.node_idx = b->d_nodes.as<int32_t>();
    g.nodes = reinterpret_cast<const float4*>(nodes_dev);
    g.n_nodes = prm->n_nodes;
    g.rec = b->packed.as<float4>();
    g.acc = reinterpret_cast<float4*>(acc_dev);
    g.G = prm->G;
    g.eps2 = prm->soft_eps * prm->soft_eps;
    g.tile = tile;
    g.order = b->d_order.as<int32_t>();
    ReorgArgs& r = sr.reorg;
    r = ReorgArgs{};
    r.U = b->d_U.as<int32_t>();
    r.u = b->u;
    r.src = p->src;
    r.pool = p->rec.as<float4>();
    r.slot_of = p->slot_of.as<int32_t>();
    r.occ = p->occ.as<uint32_t>();
    r.cap = p->cap;
    r.pack = 1;
    r.packed = b->packed.as<float4>();
    r.uslot = b->uslot.as<int32_t>();
    r.missing = b->missing.as<int32_t>();
    r.mslot = b->mslot.as<int32_t>();
    r.free_list = b->free_list.as<uint64_t>();
    r.state = b->state.as<int32_t>();
    r.nbu = union_blocks(b->u);
    // the free slots are scanned in round 0 only; later rounds read that list at an offset
    r.nbf = k == 0 ? free_blocks(p->cap) : 0;
    sr.n_chain = r.nbu + r.nbf;
    sr.prev = -1;
    for (int32_t q = k - 1; q >= 0 && sr.prev < 0; --q)
      if (rounds[q].n_chain > 0) sr.prev = q;
    // With the evicting fixture every round sees the pool as round 0 found it: a round's table part
    // leaves the chare table and occupancy as they were (it writes for its staged ids the values
    // they already hold), and the records it stages go into free slots that no lookup reads.  Its
    // reorganisation then depends only on round 0's free-slot list and count, not on any earlier
    // round's table or data parts: the rounds' reorganisations run side by side.
    if (fixture == GC_FIXTURE_EVICT_STAGED && k > 0 && rounds[0].reorg.nbf > 0) sr.prev = kPrevFreeList;
    // the evicting fixture: each round's union blocks evict what they stage (the same table updates
    // as an eviction before the next round, off its critical path); what the previous launch's last
    // round left (nothing, unless the pool was used between launches) is evicted by a kernel before
    // the launch
    r.evict_after = fixture == GC_FIXTURE_EVICT_STAGED ? 1 : 0;
    seg(kItemFree, k, r.nbf);
    seg(kItemUnion, k, r.nbu);
    if (!combined_pass && k >= kStepLead) seg(kItemForce, k - kStepLead, (int32_t)batches[k - kStepLead]->tasks.size());
  }
  if (!combined_pass)
    for (int32_t k = std::max<int32_t>(R - kStepLead, 0); k < R; ++k)
      seg(kItemForce, k, (int32_t)batches[k]->tasks.size());
  // the combined pass of the rounds schedule: every round's tasks in its launch order, rounds in
  // order, each with its round index and first packed target
  std::vector<StepItem> fitems;
  if (combined_pass) {
    for (int32_t k = 0; k < R; ++k) {
      const gc_batch fb = batches[k];
      for (size_t i = 0; i < fb->tasks.size(); ++i) {
        const int32_t t = fb->h_order[i];
        const gc_task& tk = fb->tasks[(size_t)t];
        StepItem it{};
        it.kind = k;
        it.idx = fb->h_pibeg[(size_t)t];
        it.i_begin = tk.i_begin;
        it.i_count = tk.i_count;
        it.j_first = tk.j_first;
        it.j_nranges = tk.j_nranges;
        it.n_first = tk.n_first;
        it.n_count = tk.n_count;
        fitems.push_back(it);
      }
    }
  }
  const int32_t n_ctr = kCtrStride * (kCtrRounds + 2 * R);
  // the launch's free-slot list: entries up to the most any round can reach (with the evicting
  // fixture every round reads from the start of the list, otherwise after what earlier rounds kept)
  int64_t flimit = 0;
  for (int32_t k = 0; k < R; ++k)
    flimit = fixture == GC_FIXTURE_EVICT_STAGED ? std::max<int64_t>(flimit, batches[k]->u) : flimit + batches[k]->u;
  flimit = std::min<int64_t>(flimit, p->cap);
  const int64_t fl_words = 1 + (int64_t)R + std::max<int64_t>(flimit, 1);
  const int32_t nt = (int32_t)items.size();
  hipError_t e = gr->step_items.ensure(sizeof(StepItem) * std::max<size_t>(items.size(), 1));
  if (e == hipSuccess) e = gr->step_rounds.ensure(sizeof(StepRound) * (size_t)R);
  if (e == hipSuccess) e = gr->step_ctr.ensure(sizeof(uint64_t) * (size_t)n_ctr);
  if (e == hipSuccess) e = gr->step_fl.ensure(sizeof(uint64_t) * (size_t)fl_words);
  if (e != hipSuccess) return set_err(ctx, GC_E_NOMEM, "whole-step schedule: %s", hipGetErrorString(e));
  uint64_t* fmeta = gr->step_fl.as<uint64_t>();
  for (int32_t k = 0; k < R; ++k) {
    rounds[k].reorg.free_list = fmeta + 1 + R;
    rounds[k].reorg.ftotal = fmeta;
    rounds[k].reorg.flimit = (int32_t)flimit;
  }
  std::vector<GravArgs> gargs;
  if (combined_pass) {
    for (int32_t k = 0; k < R; ++k) gargs.push_back(rounds[k].grav);
    hipError_t e2 = gr->round_items.ensure(sizeof(StepItem) * std::max<size_t>(fitems.size(), 1));
    if (e2 == hipSuccess) e2 = gr->round_args.ensure(sizeof(GravArgs) * (size_t)R);
    if (e2 != hipSuccess) return set_err(ctx, GC_E_NOMEM, "rounds schedule: %s", hipGetErrorString(e2));
    if (!fitems.empty())
      GC_HIP(ctx, hipMemcpyAsync(gr->round_items.p, fitems.data(), sizeof(StepItem) * fitems.size(),
                                 hipMemcpyHostToDevice, s));
    GC_HIP(ctx, hipMemcpyAsync(gr->round_args.p, gargs.data(), sizeof(GravArgs) * (size_t)R, hipMemcpyHostToDevice, s));
  }
  GC_HIP(ctx, hipMemcpyAsync(gr->step_items.p, items.data(), sizeof(StepItem) * items.size(), hipMemcpyHostToDevice, s));
  GC_HIP(ctx, hipMemcpyAsync(gr->step_rounds.p, rounds.data(), sizeof(StepRound) * (size_t)R, hipMemcpyHostToDevice, s));
  GC_HIP(ctx, launch_fill_i32(gr->step_ctr.as<int32_t>(), 0, 2 * (int64_t)n_ctr, s));
  GC_HIP(ctx, launch_fill_i32(gr->step_fl.as<int32_t>(), 0, 2 * fl_words, s));  // tag 0: never a launch's
  GC_HIP(ctx, hipStreamSynchronize(s));  // the host vectors go out of scope
  int per = 0;
  const int tpl = prm->targets_per_lane == 0 ? 1 : prm->targets_per_lane;
  GC_HIP(ctx, step_occupancy(order, tpl, tile, &per));
  // the reorganisation items alone (rounds schedule) are a few hundred: one block each, so that the
  // launch's ticket and exit counters see no more requests than there are items
  const int grid = combined_pass ? std::min(std::max(1, per) * ctx->n_cu, std::max(1, nt))
                                 : std::max(1, per) * ctx->n_cu;
  StepArgs a{};
  a.items = gr->step_items.as<StepItem>();
  a.n_items = nt;
  a.rounds = gr->step_rounds.as<StepRound>();
  a.n_rounds = R;
  a.ctr = gr->step_ctr.as<uint64_t>();
  a.fmeta = fmeta;
  a.spin_limit = kStepSpinLimit;
  a.fail_round = ctx->step_fail_round < R ? ctx->step_fail_round : -1;
  a.fail_spins = ctx->step_fail_spins ? ctx->step_fail_spins : kStepSpinLimit;
  a.has_force = combined_pass ? 0 : 1;
  // with the evicting fixture two graphs: one that first evicts what the last batch left staged,
  // one without that kernel (nothing staged: the host knows, gc_graph_launch picks)
  for (int v = 0; v < (fixture == GC_FIXTURE_EVICT_STAGED ? 2 : 1); ++v) {
    hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    if (fixture == GC_FIXTURE_EVICT_STAGED && v == 0) {
      const gc_batch pb = batches[R - 1];
      le = launch_evict(pb->missing.as<int32_t>(), pb->state.as<int32_t>() + GC_STATE_MISSING, std::max<int32_t>(pb->u, 1),
                        p->slot_of.as<int32_t>(), p->n_ids, p->occ.as<uint32_t>(), s);
    }
    if (le == hipSuccess)
      le = combined_pass ? launch_step_reorg(a, grid, s) : launch_step(order, tpl, a, grid, tile, s);
    if (le == hipSuccess && combined_pass)
      le = launch_grav_rounds(order, tpl, gr->round_items.as<StepItem>(), (int32_t)fitems.size(),
                              gr->round_args.as<GravArgs>(), tile, wpb, s);
    hipGraph_t g = nullptr;
    ce = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(ctx, le != hipSuccess ? le : ce, "whole-step capture");
    }
    (v == 0 ? gr->graph : gr->graph_noevict) = g;
    ce = hipGraphInstantiate(v == 0 ? &gr->exec : &gr->exec_noevict, g, nullptr, nullptr, 0);
    if (ce != hipSuccess) return hip_fail(ctx, ce, "hipGraphInstantiate");
  }
  gr->step_form = true;
  for (int32_t k = 0; k < R; ++k) {
    batches[k]->mode = GC_REORG_PACK;
    batches[k]->pool = p;
    batches[k]->rec = batches[k]->packed.as<float4>();
    gr->err_words.push_back(batches[k]->state.as<int32_t>() + GC_STATE_ERR);
  }
  return GC_OK;
}

extern "C" gc_status gc_graph_capture(gc_ctx ctx, int32_t n_steps, gc_batch* batches, gc_pool* pools,
                                      const int32_t* modes, const gc_force_params* prm, const float* nodes_dev,
                                      float* acc_dev, int32_t fixture, const int32_t* const* place_ids,
                                      const int32_t* const* place_slots, const int32_t* place_n, void* stream,
                                      gc_graph* out) {
  GC_ENTER(ctx);
  if (n_steps <= 0 || !batches || !pools || !modes || !prm || !out)
    return set_err(ctx, GC_E_INVAL, "gc_graph_capture: bad arguments");
  if (!stream) return set_err(ctx, GC_E_INVAL, "gc_graph_capture: capture needs a non-default stream");
  if (fixture < GC_FIXTURE_NONE || fixture > GC_FIXTURE_EVICT_STAGED)
    return set_err(ctx, GC_E_INVAL, "gc_graph_capture: bad fixture %d", fixture);
  for (int32_t k = 0; k < n_steps; ++k) {
    if (!batches[k] || !pools[k] || !batches[k]->committed)
      return set_err(ctx, GC_E_STATE, "gc_graph_capture: step %d batch not committed", k);
    gc_status hs = need_host_lists(batches[k], S(stream));  // the capture builds its items on the host
    if (hs != GC_OK) return hs;
    if (modes[k] == GC_REORG_SORTED && batches[k]->max_direct > kSortMax)
      return set_err(ctx, GC_E_UNSUPPORTED, "gc_graph_capture: SORTED list too long in step %d", k);
    int tile, wpb;
    gc_status st = check_prm(batches[k], prm, &tile, &wpb);
    if (st != GC_OK) return st;
    // size buffers outside the capture (allocation is not capturable)
    if (modes[k] != GC_REORG_NONE && ensure_reorg_buffers(batches[k], pools[k], modes[k], S(stream)) != hipSuccess)
      return set_err(ctx, GC_E_NOMEM, "gc_graph_capture: buffers");
    {
      // room for one queue word per aggregated launch (allocation is not capturable)
      const int64_t T = batches[k]->nt, agg = prm->aggregation > 0 && prm->aggregation < T ? prm->aggregation : T;
      const int64_t nl = T > 0 ? (T + agg - 1) / agg : 1;
      if (batches[k]->queue.ensure(sizeof(int32_t) * (size_t)(nl + 4)) != hipSuccess)
        return set_err(ctx, GC_E_NOMEM, "gc_graph_capture: queue");
    }
    if (fixture == GC_FIXTURE_EVICT_STAGED && pools[k] != pools[(k + n_steps - 1) % n_steps])
      return set_err(ctx, GC_E_INVAL, "gc_graph_capture: evicting fixture needs one pool for all steps");
    if (pools[k]->host_src)
      return set_err(ctx, GC_E_UNSUPPORTED,
                     "gc_graph_capture: step %d's pool has a host source (its staging is packed by the host per call)",
                     k);
    if (!pools[k]->src) return set_err(ctx, GC_E_STATE, "gc_graph_capture: step %d's pool has no source", k);
  }
  // every batch starts with a cleared state (so the first replay evicts nothing for the step before
  // step 0); the tags keep later replays apart without further clearing
  for (int32_t k = 0; k < n_steps; ++k)
    if (modes[k] != GC_REORG_NONE) GC_HIP(ctx, clear_reorg_state(batches[k], S(stream)));
  GC_HIP(ctx, hipStreamSynchronize(S(stream)));
  hipStream_t s = S(stream);
  if (prm->schedule == GC_SCHED_STEP || prm->schedule == GC_SCHED_ROUNDS) {
    gc_graph gs = new gc_graph_();
    gs->ctx = ctx;
    gs->pools.assign(pools, pools + n_steps);
    gs->batches.assign(batches, batches + n_steps);
    gs->fixture = fixture;
    for (DevBuf* d : gs->bufs()) d->h = &ctx->hooks;
    gc_status st = capture_step(ctx, n_steps, batches, pools, modes, prm, nodes_dev, acc_dev, fixture, s, gs,
                                prm->schedule == GC_SCHED_ROUNDS);
    if (st != GC_OK) {
      if (gs->exec) (void)hipGraphExecDestroy(gs->exec);
      if (gs->graph) (void)hipGraphDestroy(gs->graph);
      if (gs->exec_noevict) (void)hipGraphExecDestroy(gs->exec_noevict);
      if (gs->graph_noevict) (void)hipGraphDestroy(gs->graph_noevict);
      gs->step_items.release();
      gs->step_rounds.release();
      gs->step_ctr.release();
      gs->step_fl.release();
      gs->round_items.release();
      gs->round_args.release();
      delete gs;
      return st;
    }
    // the cleared states hold no missing list: nothing a replay could evict is staged
    for (int32_t k = 0; k < n_steps; ++k) batches[k]->staged_live = false;
    *out = gs;
    return GC_OK;
  }
  // The combined pass of a step reads only its batch's own buffers unless its records come from
  // the pool (address-list modes), so those passes can run on side streams and overlap the next
  // steps' reorganisations and passes; the pool-touching chain stays on the capture stream.
  bool overlap = n_steps > 1;
  for (int32_t k = 0; k < n_steps; ++k) {
    if (modes[k] == GC_REORG_INDIRECT || modes[k] == GC_REORG_SORTED) overlap = false;
    for (int32_t q = 0; q < k; ++q)
      if (batches[q] == batches[k]) overlap = false;  // a batch reused later would overwrite buffers in use
  }
  gc_graph gr = new gc_graph_();
  gr->ctx = ctx;
  gr->pools.assign(pools, pools + n_steps);
  gr->batches.assign(batches, batches + n_steps);
  gr->fixture = fixture;
  for (DevBuf* d : gr->bufs()) d->h = &ctx->hooks;
  auto cleanup = [&]() {
    for (hipEvent_t e : gr->events) (void)hipEventDestroy(e);
    for (hipStream_t q : gr->side) (void)hipStreamDestroy(q);
    delete gr;
  };
  const int n_side = overlap ? 3 : 0;
  for (int q = 0; q < n_side; ++q) {
    hipStream_t h = nullptr;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
      cleanup();
      return set_err(ctx, GC_E_HIP, "gc_graph_capture: side stream");
    }
    gr->side.push_back(h);
  }
  for (int q = 0; q < (overlap ? n_steps + n_side : 0); ++q) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return set_err(ctx, GC_E_HIP, "gc_graph_capture: event");
    }
    gr->events.push_back(e);
  }
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(ctx, e, "hipStreamBeginCapture");
  }
  gc_status st = GC_OK;
  std::vector<bool> used(n_side, false);
  auto fork_pass = [&](int32_t j) -> gc_status {
    const int q = j % n_side;
    if (hipStreamWaitEvent(gr->side[q], gr->events[j], 0) != hipSuccess)
      return set_err(ctx, GC_E_HIP, "capture: fork");
    used[q] = true;
    return launch_combined_async(batches[j], prm, nodes_dev, acc_dev, gr->side[q]);
  };
  for (int32_t k = 0; k < n_steps && st == GC_OK; ++k) {
    gc_batch b = batches[k];
    gc_pool p = pools[k];
    if (fixture == GC_FIXTURE_RESET_PLACE) {
      if (pool_reset_async(p, s) != hipSuccess) st = set_err(ctx, GC_E_HIP, "capture: pool reset");
      if (st == GC_OK && place_n && place_n[k] > 0 &&
          launch_place(place_ids[k], place_slots[k], place_n[k], p->src, false, p->rec.as<float4>(), p->slot_of.as<int32_t>(),
                       p->occ.as<uint32_t>(), s) != hipSuccess)
        st = set_err(ctx, GC_E_HIP, "capture: place");
    } else if (fixture == GC_FIXTURE_EVICT_STAGED) {
      const int32_t q = (k + n_steps - 1) % n_steps;  // the step before (cyclically, across replays)
      gc_batch pb = batches[q];
      if (modes[q] == GC_REORG_PACK || modes[q] == GC_REORG_INDIRECT || modes[q] == GC_REORG_SORTED) {
        if (launch_evict(pb->missing.as<int32_t>(), pb->state.as<int32_t>() + GC_STATE_MISSING, std::max<int32_t>(pb->u, 1),
                         p->slot_of.as<int32_t>(), p->n_ids, p->occ.as<uint32_t>(), s) != hipSuccess)
          st = set_err(ctx, GC_E_HIP, "capture: evict");
      }
    }
    if (st != GC_OK) break;
    if (modes[k] == GC_REORG_NONE) {
      b->mode = GC_REORG_NONE;
      b->pool = p;
      b->rec = p->src;
    } else {
      st = reorganize_async(b, p, modes[k], s);
      b->mode = modes[k];
      b->pool = p;
    }
    if (st != GC_OK) break;
    if (!overlap) {
      st = launch_combined_async(b, prm, nodes_dev, acc_dev, s);
      continue;
    }
    if (hipEventRecord(gr->events[k], s) != hipSuccess) {
      st = set_err(ctx, GC_E_HIP, "capture: fork");
      break;
    }
    // the combined pass of the step before goes in only now, so that in the graph each
    // reorganisation's first dependent is the next step's chain node and its pass the second:
    // the graph's launch keeps the chain on one queue and gives the passes the other queues
    if (k > 0) st = fork_pass(k - 1);
  }
  if (overlap && st == GC_OK) st = fork_pass(n_steps - 1);
  // join the side streams back into the capture stream
  for (int q = 0; q < n_side; ++q) {
    if (!used[q]) continue;
    if (hipEventRecord(gr->events[n_steps + q], gr->side[q]) != hipSuccess ||
        hipStreamWaitEvent(s, gr->events[n_steps + q], 0) != hipSuccess)
      if (st == GC_OK) st = set_err(ctx, GC_E_HIP, "capture: join");
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (st != GC_OK) {
    if (g) (void)hipGraphDestroy(g);
    cleanup();
    return st;
  }
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(ctx, e, "hipStreamEndCapture");
  }
  gr->graph = g;
  e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    gr->graph = nullptr;
    cleanup();
    return hip_fail(ctx, e, "hipGraphInstantiate");
  }
  for (int32_t k = 0; k < n_steps; ++k)
    gr->err_words.push_back(modes[k] != GC_REORG_NONE ? batches[k]->state.as<int32_t>() + GC_STATE_ERR : nullptr);
  *out = gr;
  return GC_OK;
}

extern "C" gc_status gc_graph_launch(gc_graph g, void* stream) {
  if (!g) return GC_E_INVAL;
  GC_ENTER(g->ctx);
  for (gc_pool p : g->pools) p->mirror_ok = false;
  if (g->step_form && g->fixture == GC_FIXTURE_EVICT_STAGED) {
    // the eviction kernel only removes what the last batch left staged: skipped when it left nothing
    const bool evict = g->batches.back()->staged_live || !g->exec_noevict;
    GC_HIP(g->ctx, hipGraphLaunch(evict ? g->exec : g->exec_noevict, S(stream)));
    for (gc_batch b : g->batches) b->staged_live = false;  // each round's staging is evicted in it
    return GC_OK;
  }
  GC_HIP(g->ctx, hipGraphLaunch(g->exec, S(stream)));
  // other graphs may leave their batches' staging in the pools
  for (gc_batch b : g->batches) b->staged_live = true;
  return GC_OK;
}

extern "C" gc_status gc_graph_status(gc_graph g, void* stream) {
  if (!g) return GC_E_INVAL;
  GC_ENTER(g->ctx);
  int hit = -1;
  GC_HIP(g->ctx, first_set_word(g->err_words, S(stream), &hit));
  if (hit >= 0)
    return set_err(g->ctx, GC_E_HIP, "gc_graph_status: a bounded wait gave up (step %d of the capture)", hit);
  return GC_OK;
}

extern "C" gc_status gc_graph_destroy(gc_graph g) {
  if (!g) return GC_E_INVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->exec_noevict) (void)hipGraphExecDestroy(g->exec_noevict);
  if (g->graph_noevict) (void)hipGraphDestroy(g->graph_noevict);
  for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
  for (hipStream_t q : g->side) (void)hipStreamDestroy(q);
  g->step_items.release();
  g->step_rounds.release();
  g->step_ctr.release();
  g->step_fl.release();
  delete g;
  return GC_OK;
}

// ===================================================================== autotune

// ---------------------------------------------------------------- tuning cache
// A flat JSON object of entries: {"key": {"tile": 256, ...}, ...}.  Only this layout is read.

struct TuneEntry {
  int32_t tile = 0, waves = 0, schedule = 0, tpl = 0, agg = 0;
  double ms = 0.0;
};

static bool parse_cache(const std::string& txt, std::map<std::string, TuneEntry>& out) {
  size_t i = 0;
  auto ws = [&]() { while (i < txt.size() && std::isspace((unsigned char)txt[i])) ++i; };
  auto str = [&](std::string& v) -> bool {
    ws();
    if (i >= txt.size() || txt[i] != '"') return false;
    size_t j = txt.find('"', i + 1);
    if (j == std::string::npos) return false;
    v = txt.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  };
  auto ch = [&](char want) -> bool {
    ws();
    if (i < txt.size() && txt[i] == want) {
      ++i;
      return true;
    }
    return false;
  };
  ws();
  if (i == txt.size()) return true;  // empty file: no entries
  if (!ch('{')) return false;
  if (ch('}')) return true;
  do {
    std::string key;
    if (!str(key) || !ch(':') || !ch('{')) return false;
    TuneEntry e;
    do {
      std::string f;
      if (!str(f) || !ch(':')) return false;
      ws();
      char* endp = nullptr;
      const double v = std::strtod(txt.c_str() + i, &endp);
      if (endp == txt.c_str() + i) return false;
      i = (size_t)(endp - txt.c_str());
      if (f == "tile") e.tile = (int32_t)v;
      else if (f == "waves_per_block") e.waves = (int32_t)v;
      else if (f == "schedule") e.schedule = (int32_t)v;
      else if (f == "targets_per_lane") e.tpl = (int32_t)v;
      else if (f == "aggregation") e.agg = (int32_t)v;
      else if (f == "ms") e.ms = v;
      else return false;
    } while (ch(','));
    if (!ch('}')) return false;
    out[key] = e;
  } while (ch(','));
  return ch('}');
}

static bool write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) {
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "  \"%s\": {\"tile\": %d, \"waves_per_block\": %d, \"schedule\": %d, \"targets_per_lane\": %d, "
                 "\"aggregation\": %d, \"ms\": %.6f}%s\n",
                 kv.first.c_str(), e.tile, e.waves, e.schedule, e.tpl, e.agg, e.ms, ++k < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// The cache key of a batch: device, force kind and a 64-bit FNV-1a hash of the batch's shape.
static std::string tune_key(gc_batch b, const gc_force_params* base) {
  hipDeviceProp_t pr;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&pr, b->ctx->device) == hipSuccess) arch = pr.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (uint64_t)((v >> (8 * k)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(b->nt);
  mix(b->n_targets);
  mix(b->n_direct);
  mix(b->nn);
  int64_t hist[8] = {0};  // tasks by target count: 1, 2-3, 4-7, ..., 64-127, >= 128
  for (const gc_task& t : b->tasks) {
    int k = 0;
    while (k < 7 && (1 << (k + 1)) <= t.i_count) ++k;
    ++hist[k];
  }
  for (int64_t v : hist) mix(v);
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s:%dcu:%s:%016llx", arch.c_str(), b->ctx->n_cu,
                base->kind == GC_FORCE_GRAV_QUAD ? "grav_quad" : "grav_mono", (unsigned long long)h);
  return buf;
}

extern "C" gc_status gc_autotune(gc_batch b, const gc_force_params* base, const float* nodes_dev, float* acc_dev,
                                 int32_t reps, float* times_ms, gc_force_params* best, const char* cache_path,
                                 int32_t* from_cache, void* stream) {
  if (!b) return GC_E_INVAL;
  gc_ctx c = b->ctx;
  GC_ENTER(c);
  if (!base || !best || reps < 1) return set_err(c, GC_E_INVAL, "gc_autotune: bad arguments");
  if (b->kind != GC_KIND_GRAV) return set_err(c, GC_E_UNSUPPORTED, "gc_autotune: gravity batches only");
  if (from_cache) *from_cache = 0;
  hipStream_t s = S(stream);
  std::map<std::string, TuneEntry> cache;
  std::string key;
  if (cache_path) {
    gc_status hs = need_host_lists(b, s);  // the key hashes the task sizes
    if (hs != GC_OK) return hs;
    key = tune_key(b, base);
    if (FILE* f = std::fopen(cache_path, "r")) {
      std::string txt;
      char buf[4096];
      size_t n;
      while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
      std::fclose(f);
      if (!parse_cache(txt, cache)) return set_err(c, GC_E_INVAL, "gc_autotune: %s is not a tuning cache", cache_path);
    }
    auto it = cache.find(key);
    if (it != cache.end()) {
      *best = *base;
      best->tile = it->second.tile;
      best->waves_per_block = it->second.waves;
      best->schedule = it->second.schedule;
      best->grid_blocks = 0;
      best->targets_per_lane = it->second.tpl;
      best->aggregation = it->second.agg;
      if (from_cache) *from_cache = 1;
      return GC_OK;
    }
  }
  hipEvent_t e0, e1;
  GC_HIP(c, hipEventCreate(&e0));
  GC_HIP(c, hipEventCreate(&e1));
  float best_t = 1e30f;
  gc_status st = GC_OK;
  auto time_one = [&](const gc_force_params& p, int idx) {
    st = launch_combined_async(b, &p, nodes_dev, acc_dev, s);  // warm-up
    if (st != GC_OK) return;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == GC_OK && e == hipSuccess; ++r) st = launch_combined_async(b, &p, nodes_dev, acc_dev, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = hip_fail(c, e, "gc_autotune timing");
    if (st != GC_OK) return;
    ms /= reps;
    if (times_ms) times_ms[idx] = ms;
    if (ms < best_t) {
      best_t = ms;
      *best = p;
    }
  };
  const int tiles[3] = {128, 256, 512}, waves[3] = {2, 4, 8};
  int idx = 0;
  for (int ti = 0; ti < 3 && st == GC_OK; ++ti)
    for (int wi = 0; wi < 3 && st == GC_OK; ++wi)
      for (int sc = 0; sc < 2 && st == GC_OK; ++sc)
        for (int tp = 1; tp <= 2 && st == GC_OK; ++tp, ++idx) {
          gc_force_params p = *base;
          p.tile = tiles[ti];
          p.waves_per_block = waves[wi];
          p.schedule = sc;
          p.grid_blocks = 0;
          p.targets_per_lane = tp;
          p.aggregation = 0;
          time_one(p, idx);
        }
  if (st == GC_OK) {
    // the aggregation count, with the best shape: all tasks, then multiples of the occupancy-sized count
    const gc_force_params shape = *best;
    int per = 1;
    const int order = base->kind == GC_FORCE_GRAV_QUAD ? 2 : 1;
    const bool lists = b->mode == GC_REORG_INDIRECT || b->mode == GC_REORG_SORTED;
    hipError_t e = grav_occupancy(order, lists, shape.schedule == 1, shape.targets_per_lane == 0 ? 1 : shape.targets_per_lane,
                                  shape.tile ? shape.tile : 256, shape.waves_per_block ? shape.waves_per_block : 4, &per);
    if (e != hipSuccess) st = hip_fail(c, e, "gc_autotune occupancy");
    const int32_t occ = std::max(1, per) * c->n_cu;
    const int32_t counts[4] = {0, 2 * occ, occ, std::max(1, occ / 2)};
    for (int k = 0; k < 4 && st == GC_OK; ++k) {
      gc_force_params p = shape;
      p.aggregation = counts[k];
      time_one(p, 36 + k);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GC_OK || !cache_path) return st;
  TuneEntry te;
  te.tile = best->tile;
  te.waves = best->waves_per_block;
  te.schedule = best->schedule;
  te.tpl = best->targets_per_lane;
  te.agg = best->aggregation;
  te.ms = best_t;
  cache[key] = te;
  if (!write_cache(cache_path, cache)) return set_err(c, GC_E_INVAL, "gc_autotune: cannot write %s", cache_path);
  return GC_OK;
}

// ===================================================================== interaction lists (tree walk)

namespace {
struct ScopedBuf {  // device scratch of one call, freed on every return path
  DevBuf d;
  explicit ScopedBuf(gc_ctx c) { d.h = &c->hooks; }
  ~ScopedBuf() { d.release(); }
};
}  // namespace

// The walk proper, on scratch the caller provides: skip (int32 [n_nodes]), tot (3 int64: the two
// totals and the invalid-bucket count), and optionally each bucket's room of the count pass (sn / sr,
// nullptr: every bucket is walked twice).
static gc_status tree_walk_impl(gc_ctx c, int32_t n_nodes, const int32_t* node_range_dev,
                                const double* node_com_dev, const double* node_side_dev, const float* rec_dev,
                                int32_t n_ids, int32_t n_buckets, const int32_t* bucket_node_dev, double theta,
                                int32_t* n_first_dev, int32_t* r_first_dev, int32_t* node_idx_dev, int64_t node_cap,
                                int32_t* ranges_dev, int64_t range_cap, int64_t* totals, int32_t* skip,
                                long long* dtot, int32_t* sn, int2* sr, hipStream_t s) {
  GC_HIP(c, launch_fill_i32(reinterpret_cast<int32_t*>(dtot), 0, 6, s));
  WalkArgs a{};
  a.range = reinterpret_cast<const int2*>(node_range_dev);
  a.com = node_com_dev;
  a.side = node_side_dev;
  a.skip = skip;
  a.rec = reinterpret_cast<const float4*>(rec_dev);
  a.bucket_node = bucket_node_dev;
  a.n_nodes = n_nodes;
  a.n_buckets = n_buckets;
  a.n_ids = n_ids;
  a.theta = theta;
  a.n_first = n_first_dev;
  a.r_first = r_first_dev;
  a.node_idx = node_idx_dev;
  a.ranges = ranges_dev;
  a.bad = reinterpret_cast<unsigned long long*>(dtot + 2);
  a.sn = sn;
  a.sr = sr;
  GC_HIP(c, launch_subtree_end(a.range, n_nodes, skip, s));
  GC_HIP(c, launch_walk(false, a, s));
  GC_HIP(c, launch_scan_counts(n_first_dev, r_first_dev, n_buckets, dtot, s));
  long long h[3] = {0, 0, 0};
  GC_HIP(c, hipMemcpyAsync(h, dtot, sizeof h, hipMemcpyDeviceToHost, s));
  GC_HIP(c, hipStreamSynchronize(s));
  totals[0] = h[0];
  totals[1] = h[1];
  if (h[2] != 0) return set_err(c, GC_E_INVAL, "gc_tree_walk: %lld buckets with a leaf index or id range out of bounds", h[2]);
  if (h[0] > INT32_MAX || h[1] > INT32_MAX)
    return set_err(c, GC_E_UNSUPPORTED, "gc_tree_walk: %lld node entries / %lld ranges exceed int32 offsets", h[0], h[1]);
  if (h[0] > node_cap || h[1] > range_cap || (h[0] > 0 && !node_idx_dev) || (h[1] > 0 && !ranges_dev))
    return set_err(c, GC_E_FULL, "gc_tree_walk: need %lld node entries and %lld ranges (capacity %lld, %lld)", h[0],
                   h[1], (long long)node_cap, (long long)range_cap);
  GC_HIP(c, launch_walk_copy(a, s));
  GC_HIP(c, launch_walk(true, a, s));
  GC_HIP(c, hipStreamSynchronize(s));  // the scratch is released or reused on return
  return GC_OK;
}

// Argument checks shared by both entry points; *done is set when there is nothing to walk.
static gc_status tree_walk_args(gc_ctx c, int32_t n_nodes, const int32_t* node_range_dev, const double* node_com_dev,
                                const double* node_side_dev, const float* rec_dev, int32_t n_ids, int32_t n_buckets,
                                const int32_t* bucket_node_dev, double theta, int32_t* n_first_dev,
                                int32_t* r_first_dev, int64_t node_cap, int64_t range_cap, int64_t* totals,
                                hipStream_t s, bool* done) {
  *done = false;
  if (!totals) return set_err(c, GC_E_INVAL, "gc_tree_walk: NULL totals");
  totals[0] = totals[1] = 0;
  if (n_nodes < 0 || n_buckets < 0 || n_ids < 0 || node_cap < 0 || range_cap < 0 || !(theta >= 0.0))
    return set_err(c, GC_E_INVAL, "gc_tree_walk: negative size or theta");
  if (n_buckets > 0 && (!n_first_dev || !r_first_dev || !bucket_node_dev))
    return set_err(c, GC_E_INVAL, "gc_tree_walk: NULL bucket argument");
  if (n_nodes > 0 && (!node_range_dev || !node_com_dev || !node_side_dev || (n_ids > 0 && !rec_dev)))
    return set_err(c, GC_E_INVAL, "gc_tree_walk: NULL node argument");
  if (n_buckets == 0) {
    *done = true;
    return GC_OK;
  }
  if (n_nodes == 0) {  // no tree: every bucket's lists are empty
    GC_HIP(c, launch_fill_i32(n_first_dev, 0, (int64_t)n_buckets + 1, s));
    GC_HIP(c, launch_fill_i32(r_first_dev, 0, (int64_t)n_buckets + 1, s));
    *done = true;
  }
  return GC_OK;
}

extern "C" gc_status gc_tree_walk(gc_ctx c, int32_t n_nodes, const int32_t* node_range_dev, const double* node_com_dev,
                                  const double* node_side_dev, const float* rec_dev, int32_t n_ids, int32_t n_buckets,
                                  const int32_t* bucket_node_dev, double theta, int32_t* n_first_dev,
                                  int32_t* r_first_dev, int32_t* node_idx_dev, int64_t node_cap, int32_t* ranges_dev,
                                  int64_t range_cap, int64_t* totals, void* stream) {
  if (!c) return GC_E_INVAL;
  GC_ENTER(c);
  hipStream_t s = S(stream);
  bool done = false;
  gc_status st = tree_walk_args(c, n_nodes, node_range_dev, node_com_dev, node_side_dev, rec_dev, n_ids, n_buckets,
                                bucket_node_dev, theta, n_first_dev, r_first_dev, node_cap, range_cap, totals, s, &done);
  if (st != GC_OK || done) return st;
  ScopedBuf skip(c), tot(c);
  if (skip.d.ensure(sizeof(int32_t) * (size_t)n_nodes) != hipSuccess || tot.d.ensure(256) != hipSuccess)
    return set_err(c, GC_E_NOMEM, "gc_tree_walk: scratch");
  // room for each bucket's lists in the count pass, kept by the context (without it every bucket is
  // walked twice)
  DevBuf& keep = c->walk_keep;
  const size_t keep_n = sizeof(int32_t) * kWalkCapNodes * (size_t)n_buckets;
  const bool kept = keep.ensure(keep_n + sizeof(int2) * kWalkCapRanges * (size_t)n_buckets) == hipSuccess;
  if (!kept) (void)hipGetLastError();
  return tree_walk_impl(c, n_nodes, node_range_dev, node_com_dev, node_side_dev, rec_dev, n_ids, n_buckets,
                        bucket_node_dev, theta, n_first_dev, r_first_dev, node_idx_dev, node_cap, ranges_dev,
                        range_cap, totals, skip.d.as<int32_t>(), tot.d.as<long long>(),
                        kept ? keep.as<int32_t>() : nullptr,
                        kept ? reinterpret_cast<int2*>(keep.as<char>() + keep_n) : nullptr, s);
}

// ---------------------------------------------------------------- the walk without allocation

// Scratch of gc_tree_walk_noalloc: the totals (bytes [0, 256)), then skip (int32 per node).  One copy
// per device, held until the process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a host-side stand-in): the context looks up its device address at gc_init.
static __device__ __align__(256) unsigned char scratch[kWalkScratchBytes];

// Device address of the current device's copy of `scratch`, looked up once per device (with that
// device current) and kept for the life of the process.
static hipError_t walk_scratch_address(void** out) {
  static std::mutex mu;
  static std::map<int, void*> by_device;
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = by_device.find(dev);
  if (it != by_device.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  by_device[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

extern "C" gc_status gc_tree_walk_noalloc(gc_ctx c, int32_t n_nodes, const int32_t* node_range_dev,
                                          const double* node_com_dev, const double* node_side_dev,
                                          const float* rec_dev, int32_t n_ids, int32_t n_buckets,
                                          const int32_t* bucket_node_dev, double theta, int32_t* n_first_dev,
                                          int32_t* r_first_dev, int32_t* node_idx_dev, int64_t node_cap,
                                          int32_t* ranges_dev, int64_t range_cap, int64_t* totals, void* stream) {
  if (!c) return GC_E_INVAL;
  GC_ENTER(c);
  if (n_nodes > kWalkNoAllocMaxNodes)
    return set_err(c, GC_E_INVAL, "gc_tree_walk_noalloc: %d nodes exceed the fixed scratch (at most %d)", n_nodes,
                   kWalkNoAllocMaxNodes);
  if (!c->walk_scratch) return set_err(c, GC_E_STATE, "gc_tree_walk_noalloc: no scratch address for this device");
  hipStream_t s = S(stream);
  bool done = false;
  gc_status st = tree_walk_args(c, n_nodes, node_range_dev, node_com_dev, node_side_dev, rec_dev, n_ids, n_buckets,
                                bucket_node_dev, theta, n_first_dev, r_first_dev, node_cap, range_cap, totals, s, &done);
  if (st != GC_OK || done) return st;
  unsigned char* base = static_cast<unsigned char*>(c->walk_scratch);
  return tree_walk_impl(c, n_nodes, node_range_dev, node_com_dev, node_side_dev, rec_dev, n_ids, n_buckets,
                        bucket_node_dev, theta, n_first_dev, r_first_dev, node_idx_dev, node_cap, ranges_dev,
                        range_cap, totals, reinterpret_cast<int32_t*>(base + 256), reinterpret_cast<long long*>(base),
                        nullptr, nullptr, s);
}
