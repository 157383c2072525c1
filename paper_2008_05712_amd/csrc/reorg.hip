// Reorganisation kernels (Sec. 3.2): residency lookup of the combined
// request's union in the chare table, slot assignment and staging of missing
// records, the packing gather (or the source gather for redundant transfers),
// the address-list remaps, and eviction.
//
// The union U of a batch (sorted distinct ids over its target and direct
// ranges) and every position in it are fixed when the batch is committed: the
// host builds them once, as the runtime keeps its index lists sorted on
// insertion.  What depends on the pool's state is done here, in one launch:
//   k_reorg  blocks take tickets in dispatch order.  The first tickets scan the
//            occupancy flags for free slots (ascending), the rest look up their
//            chunk of U in slot_of.  Each side is a single-pass scan with
//            decoupled look-back; a union block then takes, for its k-th missing
//            record overall, the k-th free slot from the free-slot blocks'
//            published list, stages the record there and writes the packed
//            copy of every union entry it owns.
// Every status word and free-list entry carries the tag of the call that wrote
// it, so nothing has to be cleared between calls; the last block to finish
// advances the tag and rewinds the two counters.  Union blocks only wait on
// free-slot blocks, which hold earlier tickets and so are already running: no
// wait can depend on a block that has not been dispatched.  Every wait is
// bounded (an error flag is raised instead of hanging).
// Address lists (indirect and sorted modes) are one more coalesced pass over
// the static union ranks of the list entries, plus a per-task sort.
#include <climits>

#include "gc_internal.h"

namespace gc {
namespace {

constexpr int kRThreads = 256;
constexpr int kUItems = 8;                          // union entries per thread
constexpr int kUBlock = kRThreads * kUItems;        // union entries per block
constexpr int kFItems = 16;                         // occupancy entries per thread
constexpr int kFBlock = kRThreads * kFItems;        // pool slots per free-scan block
constexpr uint32_t kSpinLimit = 1u << 22;           // bound on every wait: each wave exits

// state[] layout (int32 units); see gc_internal.h for the host-visible part
constexpr int kTicket = 8, kDone = 9, kTag = 10, kFreeTotal = 12, kLookBack = 16;

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across the block; block total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int* sh_wave, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) sh_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    int s = sh_wave[k];
    off += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Tagged 64-bit words: bits 0-30 a count, bit 31 a flag, bits 32-63 the call tag.  Relaxed
// device-scope atomics: each word carries its own payload, nothing else is published through it
// (acquire/release here would write back and invalidate the caches on every probe).
__device__ __forceinline__ uint64_t tword(uint32_t tag, uint32_t flag, uint32_t cnt) {
  return ((uint64_t)tag << 32) | ((uint64_t)flag << 31) | (uint64_t)cnt;
}
__device__ __forceinline__ void tstore(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t tload(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t iload(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void istore(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront 0 of chain block `bid`: publish the block aggregate, look back over up to 64
// predecessors per probe (a word of another call counts as not yet written; the run up to the
// nearest inclusive prefix is summed once all of it is written), publish the inclusive prefix,
// return the exclusive prefix.
__device__ __forceinline__ uint32_t look_back(uint64_t* flags, int bid, uint32_t tag, uint32_t agg, int32_t* err) {
  const int lane = threadIdx.x & 63;
  if (bid == 0) {
    if (lane == 0) tstore(flags, tword(tag, 1, agg));
    return 0;
  }
  if (lane == 0) tstore(flags + bid, tword(tag, 0, agg));
  uint32_t x = 0, spins = 0;
  int hi = bid - 1;
  while (true) {
    const int j = hi - lane;
    const uint64_t w = j >= 0 ? tload(flags + j) : tword(tag, 1, 0);  // before block 0: a zero prefix
    const bool mine = (uint32_t)(w >> 32) == tag;
    const uint64_t pre = __ballot(mine && ((w >> 31) & 1u));
    const uint64_t emp = __ballot(!mine);
    const int stop = pre ? __builtin_ctzll(pre) : 63;  // last lane of the run to sum
    const uint64_t run = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
    if (emp & run) {
      if (++spins > kSpinLimit) {
        if (lane == 0) istore(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint32_t v = lane <= stop ? (uint32_t)(w & 0x7fffffffu) : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    x += v;
    if (pre) break;
    hi -= 64;
  }
  if (lane == 0) tstore(flags + bid, tword(tag, 1, x + agg));
  return x;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Pool reset: slot_of[0, n_ids) = -1 and occ[0, cap) = 0 in one grid.
__global__ void k_pool_reset(int32_t* __restrict__ slot_of, int32_t n_ids, uint32_t* __restrict__ occ, int32_t cap) {
  const int64_t n = n_ids > cap ? n_ids : cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n_ids) slot_of[i] = -1;
    if (i < cap) occ[i] = 0u;
  }
}

// Free-slot side: the lowest free slots in ascending order, listed up to `limit` (|U|, an upper
// bound on the number of missing records); the last block publishes the pool's free count.
__device__ __forceinline__ void free_role(const ReorgArgs& a, int b, uint32_t tag, int* sh, uint32_t* s_ex) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack);
  const int64_t s0 = (int64_t)b * kFBlock + (int64_t)threadIdx.x * kFItems;
  uint32_t f = 0;
  if (s0 < a.cap) {
    const uint4* o4 = reinterpret_cast<const uint4*>(a.occ + s0);  // occ is padded to whole blocks
#pragma unroll
    for (int q = 0; q < kFItems / 4; ++q) {
      const uint4 o = o4[q];
      const uint32_t ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (ov[k] == 0u && s0 + 4 * q + k < a.cap) f |= 1u << (4 * q + k);
    }
  }
  int tot;
  int r = block_excl_scan(__popc(f), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbf - 1) {
        tstore(reinterpret_cast<uint64_t*>(a.state + kFreeTotal), tword(tag, 0, ex + (uint32_t)tot));
        a.state[GC_STATE_FREE] = (int32_t)(ex + (uint32_t)tot);
      }
    }
  }
  __syncthreads();
  r += (int)*s_ex;
  if (r >= a.u) return;
#pragma unroll
  for (int k = 0; k < kFItems; ++k)
    if ((f >> k) & 1u) {
      if (r < a.u) tstore(a.free_list + r, tword(tag, 0, (uint32_t)(s0 + k)));
      ++r;
    }
}

// Union side: residency of this block's chunk of U, the missing ranks, then slot assignment,
// staging and the packed copies.
__device__ __forceinline__ void union_role(const ReorgArgs& a, int b, uint32_t tag, int* sh, uint32_t* s_ex) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack) + a.nbf;
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  int32_t id[kUItems], sl[kUItems];
  uint32_t fm = 0;
  {
    const int4* u4 = reinterpret_cast<const int4*>(a.U + k0);  // U is padded to whole blocks
    const int4 x = u4[0], y = u4[1];
    id[0] = x.x; id[1] = x.y; id[2] = x.z; id[3] = x.w;
    id[4] = y.x; id[5] = y.y; id[6] = y.z; id[7] = y.w;
  }
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    sl[i] = 0;
    if (k0 + i < a.u) {
      sl[i] = a.slot_of[id[i]];
      if (sl[i] < 0) fm |= 1u << i;
    }
  }
  // records of the missing entries: their loads do not wait for any rank
  float rx[kUItems], ry[kUItems], rz[kUItems], rw[kUItems];
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((fm >> i) & 1u) v = a.src[id[i]];
    rx[i] = v.x;
    ry[i] = v.y;
    rz[i] = v.z;
    rw[i] = v.w;
  }
  int tot;
  int rm = block_excl_scan(__popc(fm), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbu - 1) {
        a.state[GC_STATE_UNION] = a.u;
        a.state[GC_STATE_MISSING] = (int32_t)(ex + (uint32_t)tot);
      }
    }
  }
  // resident entries do not depend on the look-back
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    const int64_t k = k0 + i;
    if (k < a.u && !((fm >> i) & 1u)) {
      a.uslot[k] = sl[i];
      if (a.pack) a.packed[k] = a.pool[sl[i]];
    }
  }
  __syncthreads();
  if (!fm) return;
  rm += (int)*s_ex;
  // the rm-th free slot for the rm-th missing record, once its free-scan block has listed it (none if
  // the pool is full): one probe for all of this thread's entries in flight, then a bounded wait that
  // re-probes the entries still unlisted
  uint64_t w[kUItems];
  uint32_t pend = 0;
  {
    int r = rm;
#pragma unroll
    for (int i = 0; i < kUItems; ++i)
      if ((fm >> i) & 1u) {
        w[i] = tload(a.free_list + r++);
        if ((uint32_t)(w[i] >> 32) != tag) pend |= 1u << i;
      }
  }
  uint32_t spins = 0;
  while (pend) {
    if (++spins > kSpinLimit) {
      istore(a.state + GC_STATE_ERR, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    const uint64_t t = tload(reinterpret_cast<uint64_t*>(a.state + kFreeTotal));
    const bool total_known = (uint32_t)(t >> 32) == tag;
    int r = rm;
#pragma unroll
    for (int i = 0; i < kUItems; ++i)
      if ((fm >> i) & 1u) {
        if ((pend >> i) & 1u) {
          w[i] = tload(a.free_list + r);
          if ((uint32_t)(w[i] >> 32) == tag || (total_known && (uint32_t)r >= (uint32_t)(t & 0x7fffffffu)))
            pend &= ~(1u << i);
        }
        ++r;
      }
  }
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    if (!((fm >> i) & 1u)) continue;
    const int64_t k = k0 + i;
    const int32_t s = (uint32_t)(w[i] >> 32) == tag ? (int32_t)(w[i] & 0x7fffffffu) : -1;
    a.missing[rm] = id[i];
    a.mslot[rm] = s;
    a.uslot[k] = s;
    const float4 v = make_float4(rx[i], ry[i], rz[i], rw[i]);
    if (s >= 0) {
      a.pool[s] = v;
      a.slot_of[id[i]] = s;
      a.occ[s] = 1u;
    }
    if (a.pack) a.packed[k] = v;
    ++rm;
  }
}

__global__ void __launch_bounds__(kRThreads) k_reorg(ReorgArgs a) {
  __shared__ int sh[kRThreads / 64];
  __shared__ int s_ticket;
  __shared__ uint32_t s_tag, s_ex;
  if (threadIdx.x == 0) {
    s_ticket = atomicAdd(a.state + kTicket, 1);
    s_tag = (uint32_t)iload(a.state + kTag) + 1u;
  }
  __syncthreads();
  const int t = s_ticket;
  const uint32_t tag = s_tag;
  if (t < a.nbf)
    free_role(a, t, tag, sh, &s_ex);
  else
    union_role(a, t - a.nbf, tag, sh, &s_ex);
  __syncthreads();
  if (threadIdx.x == 0) {
    // the last block out rewinds the counters and makes this call's tag the current one
    if (atomicAdd(a.state + kDone, 1) == a.nbf + a.nbu - 1) {
      istore(a.state + kTicket, 0);
      istore(a.state + kDone, 0);
      istore(a.state + kTag, (int32_t)tag);
    }
  }
}

// Redundant transfers: every union record is gathered from the source, the pool is not used.
__global__ void k_gather_src(const int32_t* __restrict__ U, int32_t u, const float4* __restrict__ src,
                             float4* __restrict__ packed, int32_t* __restrict__ state) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    state[GC_STATE_UNION] = u;
    state[GC_STATE_MISSING] = u;
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < u; k += gridDim.x * blockDim.x) packed[k] = src[U[k]];
}

// Address lists from the static union ranks of their entries: slot of each entry (0 for an entry
// left without a slot by a full pool; the reorganisation reports that case).
__global__ void k_lists(const int32_t* __restrict__ irank, int64_t n_i, const int32_t* __restrict__ jrank, int64_t n_j,
                        const int32_t* __restrict__ uslot, int32_t* __restrict__ ilist, int32_t* __restrict__ jlist) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_i + n_j; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n_i) {
      const int32_t v = uslot[irank[e]];
      ilist[e] = v > 0 ? v : 0;
    } else {
      const int32_t v = uslot[jrank[e - n_i]];
      jlist[e - n_i] = v > 0 ? v : 0;
    }
  }
}

// Capacity check without side effects: out[0] += missing records of U, out[1] += free slots.
__global__ void __launch_bounds__(256) k_count(const int32_t* __restrict__ U, int32_t u,
                                               const int32_t* __restrict__ slot_of, const uint32_t* __restrict__ occ,
                                               int32_t cap, int32_t* __restrict__ out) {
  __shared__ int sh[4];
  int m = 0, f = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (u > cap ? u : cap);
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k < u && slot_of[U[k]] < 0) ++m;
    if (k < cap && occ[k] == 0u) ++f;
  }
  int tm, tf;
  (void)block_excl_scan(m, sh, &tm);
  (void)block_excl_scan(f, sh, &tf);
  if (threadIdx.x == 0) {
    if (tm) atomicAdd(out, tm);
    if (tf) atomicAdd(out + 1, tf);
  }
}

// Eviction: ids[0, n) leave the pool (n = min(*n_dev, n_host) when n_dev is given).  Ids outside
// [0, n_ids) and ids not resident are skipped.
__global__ void k_evict(const int32_t* __restrict__ ids, const int32_t* __restrict__ n_dev, int32_t n_host,
                        int32_t* __restrict__ slot_of, int32_t n_ids, uint32_t* __restrict__ occ) {
  const int32_t n = n_dev ? min(*n_dev, n_host) : n_host;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t id = ids[k];
    if (id < 0 || id >= n_ids) continue;
    const int32_t s = slot_of[id];
    if (s < 0) continue;
    slot_of[id] = -1;
    occ[s] = 0u;
  }
}

__global__ void k_place(const int32_t* __restrict__ ids, const int32_t* __restrict__ slots, int32_t n,
                        const float4* __restrict__ src, float4* __restrict__ pool, int32_t* __restrict__ slot_of,
                        uint32_t* __restrict__ occ) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    int id = ids[k], s = slots[k];
    pool[s] = src[id];
    slot_of[id] = s;
    occ[s] = 1u;
  }
}

// One block per task: ascending sort of the task's slot list in LDS (bitonic network).
__global__ void __launch_bounds__(256) k_sort_lists(int32_t n_tasks, const int32_t* __restrict__ joff,
                                                    int32_t* __restrict__ jlist) {
  __shared__ int32_t buf[kSortMax];
  for (int t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const int b = joff[t], n = joff[t + 1] - b;
    if (n <= 1) continue;
    int P = 1;
    while (P < n) P <<= 1;
    for (int k = threadIdx.x; k < P; k += blockDim.x) buf[k] = k < n ? jlist[b + k] : INT_MAX;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int k = threadIdx.x; k < P / 2; k += blockDim.x) {
          int lo = 2 * k - (k & (stride - 1));
          int hi = lo + stride;
          bool up = (lo & size) == 0;
          int x = buf[lo], y = buf[hi];
          if ((x > y) == up) {
            buf[lo] = y;
            buf[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) jlist[b + k] = buf[k];
    __syncthreads();
  }
}

inline int grid_for(int64_t n, int per_block, int cap = 65536) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int union_blocks(int32_t u) { return u > 0 ? (int)(((int64_t)u + kUBlock - 1) / kUBlock) : 1; }

int64_t union_padded(int32_t u) { return (int64_t)union_blocks(u) * kUBlock; }

int free_blocks(int32_t cap) {
  int64_t b = ((int64_t)cap + kFBlock - 1) / kFBlock;
  return b > 0 ? (int)b : 1;
}

int64_t occ_words(int32_t cap) {
  // one int per slot, padded so that every free-scan thread's 16-slot load stays inside the allocation
  return (int64_t)free_blocks(cap) * kFBlock;
}

int32_t reorg_state_ints(int32_t u, int32_t cap) { return kLookBack + 2 * (union_blocks(u) + free_blocks(cap)); }

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_pool_reset(int32_t* slot_of, int32_t n_ids, uint32_t* occ, int32_t cap, hipStream_t s) {
  int64_t n = n_ids > cap ? n_ids : cap;
  hipLaunchKernelGGL(k_pool_reset, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, slot_of, n_ids, occ, cap);
  return hipGetLastError();
}

hipError_t launch_reorg(ReorgArgs a, hipStream_t s) {
  a.nbu = union_blocks(a.u);
  a.nbf = free_blocks(a.cap);
  hipLaunchKernelGGL(k_reorg, dim3(a.nbu + a.nbf), dim3(kRThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_src(const int32_t* U, int32_t u, const float4* src, float4* packed, int32_t* state,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gather_src, dim3(grid_for(u, 256, 4096)), dim3(256), 0, s, U, u, src, packed, state);
  return hipGetLastError();
}

hipError_t launch_lists(const int32_t* irank, int64_t n_i, const int32_t* jrank, int64_t n_j, const int32_t* uslot,
                        int32_t* ilist, int32_t* jlist, hipStream_t s) {
  if (n_i + n_j <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lists, dim3(grid_for(n_i + n_j, 256, 16384)), dim3(256), 0, s, irank, n_i, jrank, n_j, uslot,
                     ilist, jlist);
  return hipGetLastError();
}

hipError_t launch_count(const int32_t* U, int32_t u, const int32_t* slot_of, const uint32_t* occ, int32_t cap,
                        int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(grid_for(u > cap ? u : cap, 256, 2048)), dim3(256), 0, s, U, u, slot_of, occ, cap,
                     out);
  return hipGetLastError();
}

hipError_t launch_evict(const int32_t* ids, const int32_t* n_dev, int32_t n_bound, int32_t* slot_of, int32_t n_ids,
                        uint32_t* occ, hipStream_t s) {
  if (n_bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_evict, dim3(grid_for(n_bound, 256, 4096)), dim3(256), 0, s, ids, n_dev, n_bound, slot_of, n_ids,
                     occ);
  return hipGetLastError();
}

hipError_t launch_sort_lists(int32_t n_tasks, const int32_t* joff, int32_t* jlist, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_lists, dim3(grid_for(n_tasks, 1, 8192)), dim3(256), 0, s, n_tasks, joff, jlist);
  return hipGetLastError();
}

hipError_t launch_place(const int32_t* ids, const int32_t* slots, int32_t n, const float4* src, float4* pool,
                        int32_t* slot_of, uint32_t* occ, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_place, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ids, slots, n, src, pool, slot_of, occ);
  return hipGetLastError();
}

}  // namespace gc
