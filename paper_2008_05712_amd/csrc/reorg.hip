// Reorganisation kernels (Sec. 3.2): residency lookup and marking, the sorted
// union of accessed ids, slot assignment and staging of missing records, the
// packing gather, and the list remaps (packed ranges, address lists, sorted
// address lists).
//
// Two launches per reorganisation:
//   k_scan   two independent single-pass scans (decoupled look-back) in one grid:
//            over the ids, each block first marking its window of 1024 ids in LDS
//            from the sorted distinct ranges of the combined request (the chare-table
//            lookup reads slot_of there): pos[id], U, the missing list, and per union rank its pool
//            slot or -(missing rank+1); over the occupancy flags: the lowest
//            free slots, ascending, up to a static bound on #missing;
//   k_apply  staging of missing records into their slots, the packing gather
//            (or the source gather for redundant transfers), and the range or
//            address-list remap, in one grid (block ranges split the roles); it
//            also clears the scan counters and look-back words for the next call.
// A per-task sort follows for sorted address lists.  All of it is HBM/L2
// bound: coalesced flag and index arrays, one 16-byte record per lane.
#include <climits>

#include "gc_internal.h"

namespace gc {
namespace {

constexpr int kLBThreads = 256;
constexpr int kLBItems = 4;
constexpr int kLBBlock = kLBThreads * kLBItems;  // ids per block
static_assert(kLBBlock == kUnionBlockIds, "host mark windows assume this block size");
constexpr uint32_t kSpinLimit = 1u << 24;       // look-back bound: every wave exits

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

// Look-back status words: bits 0-1 status (0 empty, 1 block aggregate, 2 inclusive prefix),
// bits 2-32 first count, bits 33-63 second count (each < 2^31).
__device__ __forceinline__ uint64_t lb_pack(uint32_t st, uint32_t a, uint32_t b) {
  return (uint64_t)st | ((uint64_t)a << 2) | ((uint64_t)b << 33);
}

// A status word carries its own payload, so relaxed device-scope atomics suffice (no other
// memory is published through it); acquire/release here would write back and invalidate caches.
__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront 0 of block `bid`: publish the block aggregate (a, b), look back over up to 64
// predecessors per step (one lane each: the run up to the nearest inclusive prefix is summed
// once none of it is still empty), publish the inclusive prefix.  Sets err[0] if a
// predecessor never publishes within the spin bound (not expected; keeps every wave finite).
__device__ __forceinline__ void lb_resolve(uint64_t* flags, int bid, uint32_t a, uint32_t b, uint32_t* ea,
                                           uint32_t* eb, int32_t* err) {
  const int lane = threadIdx.x & 63;
  if (bid == 0) {
    if (lane == 0) lb_store(flags, lb_pack(2, a, b));
    *ea = 0;
    *eb = 0;
    return;
  }
  if (lane == 0) lb_store(flags + bid, lb_pack(1, a, b));
  uint32_t xa = 0, xb = 0, spins = 0;
  int hi = bid - 1;
  while (true) {
    const int j = hi - lane;
    const uint64_t w = j >= 0 ? lb_load(flags + j) : lb_pack(2, 0, 0);  // before block 0: a zero prefix
    const uint32_t st = (uint32_t)(w & 3u);
    const uint64_t pre = __ballot(st == 2);
    const uint64_t emp = __ballot(st == 0);
    const int stop = pre ? __builtin_ctzll(pre) : 63;  // last lane of the run to sum
    const uint64_t run = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
    if (emp & run) {
      if (++spins > kSpinLimit) {
        if (lane == 0) err[0] = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint32_t va = lane <= stop ? (uint32_t)((w >> 2) & 0x7fffffffu) : 0u;
    uint32_t vb = lane <= stop ? (uint32_t)(w >> 33) : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      va += __shfl_xor(va, off, 64);
      vb += __shfl_xor(vb, off, 64);
    }
    xa += va;
    xb += vb;
    if (pre) break;
    hi -= 64;
  }
  if (lane == 0) lb_store(flags + bid, lb_pack(2, xa + a, xb + b));
  *ea = xa;
  *eb = xb;
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

__device__ __forceinline__ void occ_set(uint32_t* occ, int32_t s) { occ[s] = 1u; }

// Union of marked ids, position map and missing list.  counts[0] = |U|, counts[1] = #missing.
// uslot[rank] = pool slot of a resident id, or -(missing rank + 1).
__device__ __forceinline__ void union_body(const int2* __restrict__ mark, const int2* __restrict__ mwin,
                                           const int32_t* __restrict__ slot_of, int32_t n, int32_t with_missing,
                                           uint64_t* __restrict__ flags, int32_t* __restrict__ ctr,
                                           int32_t* __restrict__ pos, int32_t* __restrict__ U,
                                           int32_t* __restrict__ uslot, int32_t* __restrict__ missing,
                                           int32_t* __restrict__ counts, int nblocks) {
  __shared__ int sh[kLBThreads / 64];
  __shared__ int s_bid;
  __shared__ uint32_t s_ex[2];
  __shared__ uint32_t need[kLBBlock / 4];  // one byte per id of this block's window
  if (threadIdx.x == 0) s_bid = atomicAdd(ctr, 1);
  need[threadIdx.x] = 0u;
  __syncthreads();
  const int bid = s_bid;
  const int64_t wbase = (int64_t)bid * kLBBlock;
  // mark: the sorted distinct ranges that can reach this window are mark[mwin.x, mwin.y)
  {
    const int2 w = mwin[bid];
    uint8_t* nb = reinterpret_cast<uint8_t*>(need);
    for (int m = w.x + threadIdx.x; m < w.y; m += blockDim.x) {
      const int2 g = mark[m];
      const int64_t a = g.x > wbase ? g.x : wbase;
      const int64_t e = (int64_t)g.x + g.y < wbase + kLBBlock ? (int64_t)g.x + g.y : wbase + kLBBlock;
      for (int64_t id = a; id < e; ++id) nb[id - wbase] = 1;
    }
  }
  __syncthreads();
  const int64_t base = wbase + (int64_t)threadIdx.x * kLBItems;
  uint32_t fu = 0, fm = 0;
  int sv[4] = {-1, -1, -1, -1};
  if (base < n) {
    const uint32_t w = need[threadIdx.x];
    int4 s4 = *reinterpret_cast<const int4*>(slot_of + base);
    sv[0] = s4.x; sv[1] = s4.y; sv[2] = s4.z; sv[3] = s4.w;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (((w >> (8 * k)) & 0xffu) && base + k < n) {
        fu |= 1u << k;
        if (with_missing && sv[k] < 0) fm |= 1u << k;
      }
    }
  }
  int tu, tm;
  int ru = block_excl_scan(__popc(fu), sh, &tu);
  int rm = block_excl_scan(__popc(fm), sh, &tm);
  if (threadIdx.x < 64) {
    uint32_t ea, eb;
    lb_resolve(flags, bid, (uint32_t)tu, (uint32_t)tm, &ea, &eb, counts + 4);
    if (threadIdx.x == 0) {
      s_ex[0] = ea;
      s_ex[1] = eb;
      if (bid == nblocks - 1) {
        counts[0] = (int32_t)(ea + tu);
        counts[1] = (int32_t)(eb + tm);
      }
    }
  }
  __syncthreads();
  ru += (int)s_ex[0];
  rm += (int)s_ex[1];
  if (base >= n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t id = base + k;
    if (id >= n) break;
    if ((fu >> k) & 1u) {
      pos[id] = ru;  // only marked ids get a position; other entries are stale and never read
      U[ru] = (int32_t)id;
      if ((fm >> k) & 1u) {
        uslot[ru] = -(rm + 1);
        missing[rm++] = (int32_t)id;
      } else {
        uslot[ru] = sv[k];
      }
      ++ru;
    }
  }
}

// Free slots ascending from the occupancy flags (one int per slot, 1 = in use).
constexpr int kFreeSlotsPerBlock = kLBBlock;

__device__ __forceinline__ void free_body(const uint32_t* __restrict__ occ, int32_t cap, int32_t limit,
                                          uint64_t* __restrict__ flags, int32_t* __restrict__ ctr,
                                          int32_t* __restrict__ free_list, int32_t* __restrict__ counts, int nblocks) {
  __shared__ int sh[kLBThreads / 64];
  __shared__ int s_bid;
  __shared__ uint32_t s_ex;
  if (threadIdx.x == 0) s_bid = atomicAdd(ctr, 1);
  __syncthreads();
  const int bid = s_bid;
  const int64_t slot0 = (int64_t)bid * kFreeSlotsPerBlock + (int64_t)threadIdx.x * kLBItems;
  uint32_t f = 0;
  if (slot0 < cap) {
    const uint4 o = *reinterpret_cast<const uint4*>(occ + slot0);
    const uint32_t ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (ov[k] == 0u && slot0 + k < cap) f |= 1u << k;
  }
  const int c = __popc(f);
  int t;
  int r = block_excl_scan(c, sh, &t);
  if (threadIdx.x < 64) {
    uint32_t ea, eb;
    lb_resolve(flags, bid, (uint32_t)t, 0u, &ea, &eb, counts + 4);
    if (threadIdx.x == 0) {
      s_ex = ea;
      if (bid == nblocks - 1) counts[2] = (int32_t)(ea + t);
    }
  }
  __syncthreads();
  r += (int)s_ex;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (((f >> k) & 1u) && r < limit) free_list[r++] = (int32_t)(slot0 + k);
}

// Both scans in one grid: blocks [0, nbu) run the union chain, the rest the free-slot chain
// (listing the first `limit` free slots, a static upper bound on #missing).  The two chains
// have their own block counters and look-back words, so neither waits on the other.
__global__ void __launch_bounds__(kLBThreads) k_scan(const int2* __restrict__ mark, const int2* __restrict__ mwin,
                                                     const int32_t* __restrict__ slot_of,
                                                     int32_t n, int32_t with_missing, int nbu,
                                                     uint64_t* __restrict__ flags_u, int32_t* __restrict__ ctr_u,
                                                     int32_t* __restrict__ pos, int32_t* __restrict__ U,
                                                     int32_t* __restrict__ uslot, int32_t* __restrict__ missing,
                                                     const uint32_t* __restrict__ occ, int32_t cap, int32_t limit,
                                                     uint64_t* __restrict__ flags_f, int32_t* __restrict__ ctr_f,
                                                     int32_t* __restrict__ free_list, int32_t* __restrict__ counts) {
  if ((int)blockIdx.x < nbu)
    union_body(mark, mwin, slot_of, n, with_missing, flags_u, ctr_u, pos, U, uslot, missing, counts, nbu);
  else
    free_body(occ, cap, limit, flags_f, ctr_f, free_list, counts, (int)gridDim.x - nbu);
}

struct ApplyArgs {
  int32_t mode;
  const int32_t* counts;
  const int32_t* U;
  const int32_t* uslot;
  const int32_t* free_list;
  const int32_t* pos;
  const float4* src;
  float4* pool;
  int32_t* slot_of;
  uint32_t* occ;
  float4* packed;
  const gc_task* tasks;
  int32_t n_tasks;
  const int2* ranges;
  int32_t n_ranges;
  int2* pranges;
  int32_t* pibeg;
  const int32_t* ioff;
  const int32_t* joff;
  int32_t* ilist;
  int32_t* jlist;
  int32_t blocks_a;  // blocks [0, blocks_a) stage and pack; the rest remap
  int32_t* state;    // scan state: [8, n_state) (block counters, look-back words) is cleared here
  int32_t n_state;
};

// Pool slot of union rank p after staging (0 after a reported capacity overflow).
__device__ __forceinline__ int32_t slot_of_rank(const ApplyArgs& a, int32_t p, int32_t nfree) {
  const int32_t v = a.uslot[p];
  if (v >= 0) return v;
  const int32_t m = -v - 1;
  return m < nfree ? a.free_list[m] : 0;
}

__global__ void __launch_bounds__(256) k_apply(ApplyArgs a) {
  const int32_t nu = a.counts[0];
  const int32_t nfree = a.counts[1] < a.counts[2] ? a.counts[1] : a.counts[2];
  // the scans are done: leave their counters and look-back words cleared for the next reorganisation
  for (int i = 8 + blockIdx.x * blockDim.x + threadIdx.x; i < a.n_state; i += gridDim.x * blockDim.x) a.state[i] = 0;
  if ((int)blockIdx.x < a.blocks_a) {
    const int stride = a.blocks_a * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += stride) {
      const int32_t id = a.U[k];
      if (a.mode == GC_REORG_REDUNDANT) {
        a.packed[k] = a.src[id];
        continue;
      }
      const int32_t v = a.uslot[k];
      if (v >= 0) {
        if (a.mode == GC_REORG_PACK) a.packed[k] = a.pool[v];
      } else {
        const int32_t m = -v - 1;
        const float4 r = a.src[id];
        if (m < nfree) {
          const int32_t s = a.free_list[m];
          a.pool[s] = r;
          a.slot_of[id] = s;
          occ_set(a.occ, s);
        }
        if (a.mode == GC_REORG_PACK) a.packed[k] = r;
      }
    }
    return;
  }
  const int b = blockIdx.x - a.blocks_a, nb = gridDim.x - a.blocks_a;
  if (a.mode == GC_REORG_PACK || a.mode == GC_REORG_REDUNDANT) {
    for (int r = b * blockDim.x + threadIdx.x; r < a.n_ranges; r += nb * blockDim.x) {
      int2 g = a.ranges[r];
      a.pranges[r] = make_int2(g.y > 0 ? a.pos[g.x] : 0, g.y);
    }
    for (int t = b * blockDim.x + threadIdx.x; t < a.n_tasks; t += nb * blockDim.x) {
      const gc_task& tk = a.tasks[t];
      a.pibeg[t] = tk.i_count > 0 ? a.pos[tk.i_begin] : 0;
    }
    return;
  }
  // address lists: one wavefront per task; slots come from the union rank, so no
  // ordering with the staging writes above is needed
  const int lane = threadIdx.x & 63;
  const int waves = nb * (blockDim.x >> 6);
  for (int t = b * (blockDim.x >> 6) + (threadIdx.x >> 6); t < a.n_tasks; t += waves) {
    const gc_task tk = a.tasks[t];
    const int io = a.ioff[t];
    for (int k = lane; k < tk.i_count; k += 64) a.ilist[io + k] = slot_of_rank(a, a.pos[tk.i_begin + k], nfree);
    int o = a.joff[t];
    for (int r = 0; r < tk.j_nranges; ++r) {
      const int2 g = a.ranges[tk.j_first + r];
      for (int k = lane; k < g.y; k += 64) a.jlist[o + k] = slot_of_rank(a, a.pos[g.x + k], nfree);
      o += g.y;
    }
  }
}

__global__ void k_place(const int32_t* __restrict__ ids, const int32_t* __restrict__ slots, int32_t n,
                        const float4* __restrict__ src, float4* __restrict__ pool, int32_t* __restrict__ slot_of,
                        uint32_t* __restrict__ occ) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    int id = ids[k], s = slots[k];
    pool[s] = src[id];
    slot_of[id] = s;
    occ_set(occ, s);
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

__global__ void k_slot_to_id(const int32_t* __restrict__ slot_of, int32_t n_ids, int32_t* __restrict__ id_of_slot) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ids; i += gridDim.x * blockDim.x) {
    int s = slot_of[i];
    if (s >= 0) id_of_slot[s] = i;
  }
}

inline int grid_for(int64_t n, int per_block, int cap = 65536) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int lb_blocks(int32_t n) { return (int)((n + kLBBlock - 1) / kLBBlock) > 0 ? (int)((n + kLBBlock - 1) / kLBBlock) : 1; }

int free_blocks(int32_t cap) {
  int64_t b = ((int64_t)cap + kFreeSlotsPerBlock - 1) / kFreeSlotsPerBlock;
  return b > 0 ? (int)b : 1;
}

int64_t occ_words(int32_t cap) {
  // one int per slot, padded so that every free-scan thread's 4-slot load stays inside the allocation
  return (int64_t)free_blocks(cap) * kFreeSlotsPerBlock;
}

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

hipError_t launch_scan(const int2* mark, const int2* mwin, const int32_t* slot_of, int32_t n, int32_t with_missing,
                       uint64_t* flags_u,
                       int32_t* ctr_u, int32_t* pos, int32_t* U, int32_t* uslot, int32_t* missing, const uint32_t* occ,
                       int32_t cap, int32_t limit, uint64_t* flags_f, int32_t* ctr_f, int32_t* free_list, int32_t* counts,
                       hipStream_t s) {
  const int nbu = lb_blocks(n);
  const int nbf = with_missing ? free_blocks(cap) : 0;
  hipLaunchKernelGGL(k_scan, dim3(nbu + nbf), dim3(kLBThreads), 0, s, mark, mwin, slot_of, n, with_missing, nbu, flags_u,
                     ctr_u, pos, U, uslot, missing, occ, cap, limit, flags_f, ctr_f, free_list, counts);
  return hipGetLastError();
}

hipError_t launch_apply(int32_t mode, const int32_t* counts, int32_t bound, const int32_t* U, const int32_t* uslot,
                        const int32_t* free_list, const int32_t* pos, const float4* src, float4* pool, int32_t* slot_of,
                        uint32_t* occ, float4* packed, const gc_task* tasks, int32_t n_tasks, const int2* ranges,
                        int32_t n_ranges, int2* pranges, int32_t* pibeg, const int32_t* ioff, const int32_t* joff,
                        int32_t* ilist, int32_t* jlist, int32_t* state, int32_t n_state, hipStream_t s) {
  ApplyArgs a{mode, counts, U, uslot, free_list, pos, src, pool, slot_of, occ, packed, tasks, n_tasks, ranges,
              n_ranges, pranges, pibeg, ioff, joff, ilist, jlist, 0, state, n_state};
  a.blocks_a = grid_for(bound, 256, 4096);
  int blocks_b;
  if (mode == GC_REORG_PACK || mode == GC_REORG_REDUNDANT)
    blocks_b = grid_for(n_ranges > n_tasks ? n_ranges : n_tasks, 256, 8192);
  else
    blocks_b = grid_for(n_tasks, 4, 16384);
  hipLaunchKernelGGL(k_apply, dim3(a.blocks_a + blocks_b), dim3(256), 0, s, a);
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

hipError_t launch_slot_to_id(const int32_t* slot_of, int32_t n_ids, int32_t* id_of_slot, hipStream_t s) {
  if (n_ids <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_to_id, dim3(grid_for(n_ids, 256, 8192)), dim3(256), 0, s, slot_of, n_ids, id_of_slot);
  return hipGetLastError();
}

}  // namespace gc
