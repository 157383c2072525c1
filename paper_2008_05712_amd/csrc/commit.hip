// Device-side commit of a combined request whose tasks and lists are already on the device (from
// the list walk): validation, the per-task offsets, the union U of the request and every id's
// position in it (Sec. 3.2: the runtime keeps the request's indices sorted), the packed-space
// ranges and the longest-first launch order.  Nothing crosses to the host but a few totals.
//
// The union is built without sorting: every target and direct range adds +1 at its first id and -1
// past its last into a difference array; a prefix sum gives each id's coverage, an id is in U iff
// its coverage is positive, and a second prefix sum over those flags gives its rank.  Both prefix
// sums are block sums, one small scan of the block sums, and a rescan per block.
#include "reorg_dev.h"

namespace gc {
namespace {

constexpr int kCT = 256;                 // threads per block of the id-space kernels
constexpr int kCI = 16;                  // ids per thread
constexpr int kCB = kCT * kCI;           // ids per block
constexpr int kScanT = 1024;             // threads of the one-block scans

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per task: a task that breaks the contract is counted and emptied; otherwise its
// direct count and cost are recorded and its ranges are marked in the difference arrays (all ids
// and target ids).
__global__ void __launch_bounds__(256) k_dc_tasks(DevCommitArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= a.n_tasks) return;
  gc_task tk = a.tasks[t];
  bool bad = tk.i_count < 0 || tk.i_begin < 0 || (int64_t)tk.i_begin + tk.i_count > a.n_ids || tk.j_nranges < 0 ||
             tk.j_first < 0 || (int64_t)tk.j_first + tk.j_nranges > a.n_ranges || tk.n_count < 0 || tk.n_first < 0 ||
             (int64_t)tk.n_first + tk.n_count > a.n_node_refs || tk.flags != 0 || tk.shift[0] != 0.f ||
             tk.shift[1] != 0.f || tk.shift[2] != 0.f;
  int64_t d = 0;
  int32_t nmax = -1;
  if (!bad) {
    for (int r = lane; r < tk.j_nranges; r += 64) {
      const int2 g = a.ranges[tk.j_first + r];
      bool b = g.x < 0 || g.y < 0 || (int64_t)g.x + g.y > a.n_ids;
      if (r > 0) {
        const int2 p = a.ranges[tk.j_first + r - 1];
        b = b || (int64_t)p.x + p.y > g.x;  // ascending and disjoint
      }
      bad = bad || b;
      d += g.y;
    }
    for (int k = lane; k < tk.n_count; k += 64) {
      const int32_t nd = a.nodes[tk.n_first + k];
      bad = bad || nd < 0 || nd >= a.n_nodes;
      nmax = max(nmax, nd);
    }
  }
  bad = __ballot(bad) != 0ull;
  d = wave_sum64(d);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, 64));
  if (bad) {
    if (lane == 0) {
      atomicAdd(reinterpret_cast<unsigned long long*>(a.tot + kDcBad), 1ull);
      tk.i_count = 0;
      tk.j_nranges = 0;
      tk.n_count = 0;
      a.tasks[t] = tk;
      a.dc[t] = 0;
      a.cost[t] = 0;
    }
    return;
  }
  if (lane == 0) {
    a.dc[t] = (int32_t)min<int64_t>(d, INT32_MAX);
    a.cost[t] = (int64_t)tk.i_count * (31 * (int64_t)tk.n_count + 12 * d);
    atomicMax(reinterpret_cast<unsigned long long*>(a.tot + kDcMaxDirect), (unsigned long long)d);
    if (nmax >= 0) atomicMax(reinterpret_cast<unsigned long long*>(a.tot + kDcMaxNode), (unsigned long long)nmax);
    if (tk.i_count > 0) {
      atomicAdd(a.diff + 2 * tk.i_begin, 1);
      atomicAdd(a.diff + 2 * (tk.i_begin + tk.i_count), -1);
      atomicAdd(a.diff + 2 * tk.i_begin + 1, 1);
      atomicAdd(a.diff + 2 * (tk.i_begin + tk.i_count) + 1, -1);
    }
  }
  for (int r = lane; r < tk.j_nranges; r += 64) {
    const int2 g = a.ranges[tk.j_first + r];
    if (g.y > 0) {
      atomicAdd(a.diff + 2 * g.x, 1);
      atomicAdd(a.diff + 2 * (g.x + g.y), -1);
    }
  }
}

// Per block of kCB ids: the sums of both difference arrays (all ids, target ids).
__global__ void __launch_bounds__(kCT) k_dc_bsum(DevCommitArgs a) {
  __shared__ int sh[kCT / 64];
  const int64_t i0 = (int64_t)blockIdx.x * kCB + (int64_t)threadIdx.x * kCI;
  int sa = 0, st = 0;
  for (int k = 0; k < kCI; ++k)
    if (i0 + k <= a.n_ids) {
      const int2 v = reinterpret_cast<const int2*>(a.diff)[i0 + k];
      sa += v.x;
      st += v.y;
    }
  int ta, tt;
  (void)dev::block_excl_scan(sa, sh, &ta);
  (void)dev::block_excl_scan(st, sh, &tt);
  if (threadIdx.x == 0) {
    a.bs[2 * blockIdx.x] = ta;
    a.bs[2 * blockIdx.x + 1] = tt;
  }
}

// One block: exclusive scan in place of n values at stride `stride` (pairs scan both columns);
// the total of column c goes to tot[tot_idx + c] when tot_idx >= 0.
__global__ void __launch_bounds__(kScanT) k_dc_scan(int32_t* v, int32_t n, int32_t stride, int64_t* tot, int tot_idx) {
  __shared__ int sh[kScanT / 64];
  for (int c = 0; c < stride; ++c) {
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += kScanT) {
      const int64_t k = base + threadIdx.x;
      const int x = k < n ? v[k * stride + c] : 0;
      int t;
      const int ex = dev::block_excl_scan(x, sh, &t);
      if (k < n) v[k * stride + c] = (int32_t)(carry + ex);
      carry += t;
    }
    if (threadIdx.x == 0 && tot_idx >= 0) tot[tot_idx + c] = carry;
  }
}

// Coverage of this thread's ids from the scanned block sums: returns the all-ids coverage before
// each id (cov_a) and flags ids covered by two target ranges.
template <bool EMIT>
__device__ __forceinline__ void dc_cover(const DevCommitArgs& a, int* sh, int* s_cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * kCB + (int64_t)threadIdx.x * kCI;
  int2 v[kCI];
  int sa = 0, st = 0;
#pragma unroll
  for (int k = 0; k < kCI; ++k) {
    v[k] = i0 + k <= a.n_ids ? reinterpret_cast<const int2*>(a.diff)[i0 + k] : make_int2(0, 0);
    sa += v[k].x;
    st += v[k].y;
  }
  int ta, tt;
  int ca = dev::block_excl_scan(sa, sh, &ta) + a.bs[2 * blockIdx.x];
  int ct = dev::block_excl_scan(st, sh, &tt) + a.bs[2 * blockIdx.x + 1];
  uint32_t need = 0;
  int over = 0;
#pragma unroll
  for (int k = 0; k < kCI; ++k) {
    ca += v[k].x;
    ct += v[k].y;
    if (i0 + k < a.n_ids) {
      if (ca > 0) need |= 1u << k;
      if (ct > 1) ++over;
    }
  }
  int tn;
  int rank = dev::block_excl_scan(__popc(need), sh, &tn);
  if (!EMIT) {
    int to;
    (void)dev::block_excl_scan(over, sh, &to);
    if (threadIdx.x == 0) {
      a.ns[blockIdx.x] = tn;
      if (to) atomicAdd(reinterpret_cast<unsigned long long*>(a.tot + kDcBadTargets), (unsigned long long)to);
    }
    return;
  }
  rank += a.ns[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kCI; ++k) {
    const int64_t id = i0 + k;
    if (id >= a.n_ids) break;
    if ((need >> k) & 1u) {
      a.pos[id] = rank;
      a.U[rank] = (int32_t)id;
      ++rank;
    } else {
      a.pos[id] = -1;
    }
  }
  (void)s_cnt;
}

__global__ void __launch_bounds__(kCT) k_dc_need(DevCommitArgs a) {
  __shared__ int sh[kCT / 64];
  dc_cover<false>(a, sh, nullptr);
}

__global__ void __launch_bounds__(kCT) k_dc_emit(DevCommitArgs a) {
  __shared__ int sh[kCT / 64];
  dc_cover<true>(a, sh, nullptr);
}

// Packed-space ranges and first targets (positions in U).
__global__ void k_dc_maps(DevCommitArgs a) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (int64_t)a.n_ranges + a.n_tasks;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k < a.n_ranges) {
      const int2 g = a.ranges[k];
      const bool ok = g.y > 0 && g.x >= 0 && (int64_t)g.x + g.y <= a.n_ids;
      a.pranges[k] = make_int2(ok ? a.pos[g.x] : 0, g.y);
    } else {
      const gc_task tk = a.tasks[k - a.n_ranges];
      a.pibeg[k - a.n_ranges] = tk.i_count > 0 ? a.pos[tk.i_begin] : 0;
    }
  }
}

// One block: ioff = exclusive scan of i_count (n_tasks entries), joff = exclusive scan of the
// direct counts (n_tasks + 1 entries); totals of both.
__global__ void __launch_bounds__(kScanT) k_dc_offsets(DevCommitArgs a) {
  __shared__ int sh[kScanT / 64];
  int64_t ci = 0, cj = 0;
  for (int64_t base = 0; base < a.n_tasks; base += kScanT) {
    const int64_t t = base + threadIdx.x;
    const int xi = t < a.n_tasks ? a.tasks[t].i_count : 0;
    const int xj = t < a.n_tasks ? a.dc[t] : 0;
    int ti, tj;
    const int ei = dev::block_excl_scan(xi, sh, &ti);
    const int ej = dev::block_excl_scan(xj, sh, &tj);
    if (t < a.n_tasks) {
      a.ioff[t] = (int32_t)(ci + ei);
      a.joff[t] = (int32_t)(cj + ej);
    }
    ci += ti;
    cj += tj;
  }
  if (threadIdx.x == 0) {
    a.joff[a.n_tasks] = (int32_t)cj;
    a.tot[kDcTargets] = ci;
    a.tot[kDcDirect] = cj;
  }
}

// Longest first within each run of kLptChunk consecutive tasks, ties in task order: one block per
// run sorts (cost descending, index ascending) keys in LDS with a bitonic network.
__global__ void __launch_bounds__(1024) k_dc_order(DevCommitArgs a) {
  extern __shared__ unsigned long long key[];
  const int64_t c0 = (int64_t)blockIdx.x * kLptChunk;
  const int n = (int)min<int64_t>(kLptChunk, a.n_tasks - c0);
  int P = 1;
  while (P < n) P <<= 1;
  constexpr unsigned long long kCostMax = (1ull << 51) - 1ull;
  for (int k = threadIdx.x; k < P; k += blockDim.x) {
    if (k < n) {
      const unsigned long long c = (unsigned long long)min<int64_t>(a.cost[c0 + k], (int64_t)kCostMax);
      key[k] = ((kCostMax - c) << 13) | (unsigned long long)k;
    } else {
      key[k] = ~0ull;
    }
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = threadIdx.x; k < P / 2; k += blockDim.x) {
        const int lo = 2 * k - (k & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long x = key[lo], y = key[hi];
        if ((x > y) == up) {
          key[lo] = y;
          key[hi] = x;
        }
      }
      __syncthreads();
    }
  for (int k = threadIdx.x; k < n; k += blockDim.x) a.order[c0 + k] = (int32_t)(c0 + (int64_t)(key[k] & 8191ull));
}

// Tasks of buckets [b0, b1) from the list walk's offsets (lists relative to bucket b0's).
__global__ void k_walk_tasks(int32_t b0, int32_t b1, const int32_t* __restrict__ bucket_node, int32_t n_nodes,
                             const int2* __restrict__ node_range, const int32_t* __restrict__ n_first,
                             const int32_t* __restrict__ r_first, gc_task* __restrict__ out) {
  const int32_t nb0 = n_first[b0], rb0 = r_first[b0];
  for (int64_t b = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < b1; b += (int64_t)gridDim.x * blockDim.x) {
    gc_task t{};
    const int32_t nd = bucket_node[b];
    if (nd >= 0 && nd < n_nodes) {
      const int2 r = node_range[nd];
      t.i_begin = r.x;
      t.i_count = r.y;
    } else {
      t.i_count = -1;  // refused at commit
    }
    t.j_first = r_first[b] - rb0;
    t.j_nranges = r_first[b + 1] - r_first[b];
    t.n_first = n_first[b] - nb0;
    t.n_count = n_first[b + 1] - n_first[b];
    out[b - b0] = t;
  }
}

inline int grid_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

int dc_id_blocks(int32_t n_ids) { return (int)(((int64_t)n_ids + 1 + kCB - 1) / kCB); }

hipError_t launch_dev_commit(const DevCommitArgs& a, hipStream_t s) {
  const int nb = dc_id_blocks(a.n_ids);
  if (a.n_tasks > 0) hipLaunchKernelGGL(k_dc_tasks, dim3(grid_for(a.n_tasks, 4, 1 << 30)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_dc_bsum, dim3(nb), dim3(kCT), 0, s, a);
  hipLaunchKernelGGL(k_dc_scan, dim3(1), dim3(kScanT), 0, s, a.bs, nb, 2, a.tot, -1);
  hipLaunchKernelGGL(k_dc_need, dim3(nb), dim3(kCT), 0, s, a);
  hipLaunchKernelGGL(k_dc_scan, dim3(1), dim3(kScanT), 0, s, a.ns, nb, 1, a.tot, kDcUnion);
  hipLaunchKernelGGL(k_dc_emit, dim3(nb), dim3(kCT), 0, s, a);
  if ((int64_t)a.n_ranges + a.n_tasks > 0)
    hipLaunchKernelGGL(k_dc_maps, dim3(grid_for((int64_t)a.n_ranges + a.n_tasks, 256, 16384)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_dc_offsets, dim3(1), dim3(kScanT), 0, s, a);
  if (a.n_tasks > 0)
    hipLaunchKernelGGL(k_dc_order, dim3((a.n_tasks + kLptChunk - 1) / kLptChunk), dim3(1024),
                       sizeof(unsigned long long) * kLptChunk, s, a);
  return hipGetLastError();
}

hipError_t launch_walk_tasks(int32_t b0, int32_t b1, const int32_t* bucket_node, int32_t n_nodes,
                             const int32_t* node_range, const int32_t* n_first, const int32_t* r_first, gc_task* out,
                             hipStream_t s) {
  if (b1 <= b0) return hipSuccess;
  hipLaunchKernelGGL(k_walk_tasks, dim3(grid_for(b1 - b0, 256, 4096)), dim3(256), 0, s, b0, b1, bucket_node, n_nodes,
                     reinterpret_cast<const int2*>(node_range), n_first, r_first, out);
  return hipGetLastError();
}

}  // namespace gc
