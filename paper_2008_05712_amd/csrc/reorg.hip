// Reorganisation kernels (Sec. 3.2): residency lookup and marking, the sorted
// union of accessed ids, slot assignment and staging of missing records, the
// packing gather, and the list remaps (packed ranges, address lists, sorted
// address lists).  All kernels are plain HBM/L2-bound passes: coalesced reads
// of flag arrays, one 16-byte record per lane for the copies.
#include <climits>

#include "gc_internal.h"

namespace gc {
namespace {

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across a block of kScanThreads; returns the
// thread's exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int* sh_wave, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) sh_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    int s = sh_wave[k];
    off += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// One wavefront per range: need[id] = 1 for every id of the range.
__global__ void k_mark(const int2* __restrict__ mark, int32_t n_mark, uint8_t* __restrict__ need) {
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n_mark; r += waves) {
    int2 g = mark[r];
    for (int k = lane; k < g.y; k += 64) need[g.x + k] = 1;
  }
}

// Per-thread flags of ids [16 t, 16 t + 16): bit k of the union mask and of the missing mask.
struct IdFlags {
  uint32_t u, m;
};

__device__ __forceinline__ IdFlags load_flags(const uint8_t* __restrict__ need, const int32_t* __restrict__ slot_of,
                                              int32_t n, int64_t base, int with_missing) {
  IdFlags f{0u, 0u};
  if (base >= n) return f;
  uint4 nb = *reinterpret_cast<const uint4*>(need + base);
  uint32_t w[4] = {nb.x, nb.y, nb.z, nb.w};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    uint32_t b = (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
    if (b && base + k < n) f.u |= 1u << k;
  }
  if (with_missing && f.u) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int4 s = *reinterpret_cast<const int4*>(slot_of + base + 4 * q);
      int sv[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (((f.u >> (4 * q + k)) & 1u) && sv[k] < 0) f.m |= 1u << (4 * q + k);
    }
  }
  return f;
}

__global__ void __launch_bounds__(kScanThreads) k_union_count(const uint8_t* __restrict__ need,
                                                              const int32_t* __restrict__ slot_of, int32_t n,
                                                              int32_t with_missing, int32_t* __restrict__ bsum) {
  __shared__ int sh[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  IdFlags f = load_flags(need, slot_of, n, base, with_missing);
  int tu, tm;
  block_excl_scan(__popc(f.u), sh, &tu);
  block_excl_scan(__popc(f.m), sh, &tm);
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = tu;
    bsum[2 * blockIdx.x + 1] = tm;
  }
}

// Exclusive scan, in place, of nb (a, b) pairs by one block; totals to out[0], out[1].
__global__ void __launch_bounds__(kScanThreads) k_scan_pairs(int32_t* __restrict__ bsum, int32_t nb,
                                                             int32_t* __restrict__ out) {
  __shared__ int sh[kScanThreads / 64];
  int carry_a = 0, carry_b = 0;
  for (int32_t c = 0; c < nb; c += kScanThreads) {
    int i = c + threadIdx.x;
    int a = i < nb ? bsum[2 * i] : 0, b = i < nb ? bsum[2 * i + 1] : 0;
    int ta, tb;
    int ea = block_excl_scan(a, sh, &ta);
    int eb = block_excl_scan(b, sh, &tb);
    if (i < nb) {
      bsum[2 * i] = carry_a + ea;
      bsum[2 * i + 1] = carry_b + eb;
    }
    carry_a += ta;
    carry_b += tb;
  }
  if (threadIdx.x == 0) {
    out[0] = carry_a;
    out[1] = carry_b;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_union_write(uint8_t* __restrict__ need,
                                                              const int32_t* __restrict__ slot_of, int32_t n,
                                                              int32_t with_missing, const int32_t* __restrict__ bsum,
                                                              int32_t* __restrict__ pos, int32_t* __restrict__ U,
                                                              int32_t* __restrict__ missing) {
  __shared__ int sh[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  IdFlags f = load_flags(need, slot_of, n, base, with_missing);
  int tu, tm;
  int ru = block_excl_scan(__popc(f.u), sh, &tu) + bsum[2 * blockIdx.x];
  int rm = block_excl_scan(__popc(f.m), sh, &tm) + bsum[2 * blockIdx.x + 1];
  if (base >= n) return;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    int64_t id = base + k;
    if (id >= n) break;
    if ((f.u >> k) & 1u) {
      pos[id] = ru;
      U[ru++] = (int32_t)id;
      if ((f.m >> k) & 1u) missing[rm++] = (int32_t)id;
    } else {
      pos[id] = -1;
    }
  }
  // leave the flags cleared for the next reorganisation
  *reinterpret_cast<uint4*>(need + base) = make_uint4(0u, 0u, 0u, 0u);
}

// Free slots: flag = occ[s] == 0; the first counts[1] free slots, ascending, go to free_list.
__device__ __forceinline__ uint32_t load_free(const int32_t* __restrict__ occ, int32_t cap, int64_t base) {
  uint32_t f = 0;
  if (base >= cap) return f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int4 o = *reinterpret_cast<const int4*>(occ + base + 4 * q);
    int ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (ov[k] == 0 && base + 4 * q + k < cap) f |= 1u << (4 * q + k);
  }
  return f;
}

__global__ void __launch_bounds__(kScanThreads) k_free_count(const int32_t* __restrict__ occ, int32_t cap,
                                                             const int32_t* __restrict__ counts,
                                                             int32_t* __restrict__ bsum) {
  __shared__ int sh[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  uint32_t f = counts[1] > 0 ? load_free(occ, cap, base) : 0u;
  int t;
  block_excl_scan(__popc(f), sh, &t);
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = t;
    bsum[2 * blockIdx.x + 1] = 0;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_free_write(const int32_t* __restrict__ occ, int32_t cap,
                                                             const int32_t* __restrict__ counts,
                                                             const int32_t* __restrict__ bsum,
                                                             int32_t* __restrict__ free_list) {
  __shared__ int sh[kScanThreads / 64];
  const int need = counts[1];
  if (need == 0 || bsum[2 * blockIdx.x] >= need) return;  // uniform per block
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  uint32_t f = load_free(occ, cap, base);
  int t;
  int r = block_excl_scan(__popc(f), sh, &t) + bsum[2 * blockIdx.x];
  for (int k = 0; k < 16 && r < need; ++k)
    if ((f >> k) & 1u) free_list[r++] = (int32_t)(base + k);
}

// Stage the k-th missing record into the k-th free slot.  If the pool has fewer free
// slots than missing records (counts[1] > counts[2]) only the first counts[2] are
// staged and counts[3] is set; the others stay non-resident.
__global__ void k_stage(const int32_t* __restrict__ missing, const int32_t* __restrict__ free_list,
                        int32_t* __restrict__ counts, const float4* __restrict__ src, float4* __restrict__ pool,
                        int32_t* __restrict__ slot_of, int32_t* __restrict__ occ) {
  const int nm = counts[1] < counts[2] ? counts[1] : counts[2];
  if (blockIdx.x == 0 && threadIdx.x == 0 && counts[1] > counts[2]) counts[3] = 1;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nm; k += gridDim.x * blockDim.x) {
    int id = missing[k], s = free_list[k];
    pool[s] = src[id];
    slot_of[id] = s;
    occ[s] = 1;
  }
}

__global__ void k_place(const int32_t* __restrict__ ids, const int32_t* __restrict__ slots, int32_t n,
                        const float4* __restrict__ src, float4* __restrict__ pool, int32_t* __restrict__ slot_of,
                        int32_t* __restrict__ occ) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    int id = ids[k], s = slots[k];
    pool[s] = src[id];
    slot_of[id] = s;
    occ[s] = 1;
  }
}

__global__ void k_gather(const int32_t* __restrict__ U, const int32_t* __restrict__ counts,
                         const int32_t* __restrict__ slot_of, const float4* __restrict__ pool,
                         float4* __restrict__ packed) {
  const int nu = counts[0];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += gridDim.x * blockDim.x) {
    int s = slot_of[U[k]];  // < 0 only after a reported capacity overflow
    packed[k] = s >= 0 ? pool[s] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__global__ void k_gather_src(const int32_t* __restrict__ U, const int32_t* __restrict__ counts,
                             const float4* __restrict__ src, float4* __restrict__ packed) {
  const int nu = counts[0];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += gridDim.x * blockDim.x) packed[k] = src[U[k]];
}

__global__ void k_remap_ranges(const int2* __restrict__ ranges, int32_t n_ranges, const gc_task* __restrict__ tasks,
                               int32_t n_tasks, const int32_t* __restrict__ pos, int2* __restrict__ pranges,
                               int32_t* __restrict__ pibeg) {
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_ranges; r += stride) {
    int2 g = ranges[r];
    pranges[r] = make_int2(g.y > 0 ? pos[g.x] : 0, g.y);
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tasks; t += stride) {
    const gc_task& tk = tasks[t];
    pibeg[t] = tk.i_count > 0 ? pos[tk.i_begin] : 0;
  }
}

// One wavefront per task: pool slots of its targets and of its direct ids in list order.
__global__ void k_remap_lists(const gc_task* __restrict__ tasks, int32_t n_tasks, const int2* __restrict__ ranges,
                              const int32_t* __restrict__ ioff, const int32_t* __restrict__ joff,
                              const int32_t* __restrict__ slot_of, int32_t* __restrict__ ilist,
                              int32_t* __restrict__ jlist) {
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < n_tasks; t += waves) {
    const gc_task tk = tasks[t];
    int io = ioff[t];
    // a slot < 0 exists only after a reported capacity overflow; keep every address valid
    for (int k = lane; k < tk.i_count; k += 64) ilist[io + k] = max(slot_of[tk.i_begin + k], 0);
    int o = joff[t];
    for (int r = 0; r < tk.j_nranges; ++r) {
      int2 g = ranges[tk.j_first + r];
      for (int k = lane; k < g.y; k += 64) jlist[o + k] = max(slot_of[g.x + k], 0);
      o += g.y;
    }
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

hipError_t launch_mark(const int2* mark, int32_t n_mark, uint8_t* need, hipStream_t s) {
  if (n_mark <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark, dim3(grid_for(n_mark, 4, 16384)), dim3(256), 0, s, mark, n_mark, need);
  return hipGetLastError();
}

hipError_t launch_union_scan(const uint8_t* need, const int32_t* slot_of, int32_t n, int32_t with_missing,
                             int32_t* bsum, int32_t* pos, int32_t* U, int32_t* missing, int32_t* counts,
                             hipStream_t s) {
  int nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_union_count, dim3(nb), dim3(kScanThreads), 0, s, need, slot_of, n, with_missing, bsum);
  hipLaunchKernelGGL(k_scan_pairs, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, counts);
  hipLaunchKernelGGL(k_union_write, dim3(nb), dim3(kScanThreads), 0, s, const_cast<uint8_t*>(need), slot_of, n,
                     with_missing, bsum, pos, U, missing);
  return hipGetLastError();
}

hipError_t launch_free_scan(const int32_t* occ, int32_t cap, const int32_t* counts, int32_t* bsum,
                            int32_t* free_list, int32_t* free_count, hipStream_t s) {
  int nb = (cap + kScanBlock - 1) / kScanBlock;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_free_count, dim3(nb), dim3(kScanThreads), 0, s, occ, cap, counts, bsum);
  hipLaunchKernelGGL(k_scan_pairs, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, free_count);
  hipLaunchKernelGGL(k_free_write, dim3(nb), dim3(kScanThreads), 0, s, occ, cap, counts, bsum, free_list);
  return hipGetLastError();
}

hipError_t launch_stage(const int32_t* missing, const int32_t* free_list, int32_t* counts, int32_t bound,
                        const float4* src, float4* pool, int32_t* slot_of, int32_t* occ, hipStream_t s) {
  hipLaunchKernelGGL(k_stage, dim3(grid_for(bound, 256, 4096)), dim3(256), 0, s, missing, free_list, counts, src, pool,
                     slot_of, occ);
  return hipGetLastError();
}

hipError_t launch_place(const int32_t* ids, const int32_t* slots, int32_t n, const float4* src, float4* pool,
                        int32_t* slot_of, int32_t* occ, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_place, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ids, slots, n, src, pool, slot_of, occ);
  return hipGetLastError();
}

hipError_t launch_gather(const int32_t* U, const int32_t* counts, int32_t bound, const int32_t* slot_of,
                         const float4* pool, float4* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(grid_for(bound, 256, 8192)), dim3(256), 0, s, U, counts, slot_of, pool, packed);
  return hipGetLastError();
}

hipError_t launch_gather_src(const int32_t* U, const int32_t* counts, int32_t bound, const float4* src,
                             float4* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_src, dim3(grid_for(bound, 256, 8192)), dim3(256), 0, s, U, counts, src, packed);
  return hipGetLastError();
}

hipError_t launch_remap_ranges(const int2* ranges, int32_t n_ranges, const gc_task* tasks, int32_t n_tasks,
                               const int32_t* pos, int2* pranges, int32_t* pibeg, hipStream_t s) {
  int n = n_ranges > n_tasks ? n_ranges : n_tasks;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_remap_ranges, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, ranges, n_ranges, tasks, n_tasks,
                     pos, pranges, pibeg);
  return hipGetLastError();
}

hipError_t launch_remap_lists(const gc_task* tasks, int32_t n_tasks, const int2* ranges, const int32_t* ioff,
                              const int32_t* joff, const int32_t* slot_of, int32_t* ilist, int32_t* jlist,
                              int32_t sorted, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_remap_lists, dim3(grid_for(n_tasks, 4, 16384)), dim3(256), 0, s, tasks, n_tasks, ranges, ioff,
                     joff, slot_of, ilist, jlist);
  if (sorted) hipLaunchKernelGGL(k_sort_lists, dim3(grid_for(n_tasks, 1, 8192)), dim3(256), 0, s, n_tasks, joff, jlist);
  return hipGetLastError();
}

hipError_t launch_slot_to_id(const int32_t* slot_of, int32_t n_ids, int32_t* id_of_slot, hipStream_t s) {
  if (n_ids <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_to_id, dim3(grid_for(n_ids, 256, 8192)), dim3(256), 0, s, slot_of, n_ids, id_of_slot);
  return hipGetLastError();
}

}  // namespace gc
