// Barnes-Hut interaction lists of the buckets' work requests (Sec. 4.1: a bucket's particles share
// one node list and one direct list), built on the device.
//
// Opening test (FP64, no contraction, correctly rounded square root): bucket B takes node N when
// theta > 0, N's id range does not overlap B's and side(N) < theta * dist(com(N), box(B)); box(B) is
// the tight bounding box of B's FP32 positions and dist the distance from a point to the box, per
// axis e = lo - c below, c - hi above, else 0, summed as (e_x^2 + e_y^2) + e_z^2.  A node that is not
// taken goes, if a leaf, to the direct list as its id range and is otherwise opened.
//
// Nodes are numbered in pre-order with every node's ids contiguous, so a node's subtree is the
// index range [k, skip[k]) and the walk is one forward pass over the indices: a taken node or a leaf
// continues at skip[k], an opened node at k + 1.  Every step moves forward, so each lane ends within
// n_nodes steps.  One lane per bucket.  The count pass also keeps each bucket's lists, up to a fixed
// room; after the scan of the counts they are copied to their offsets, and only a bucket that did
// not fit is walked again.
#include "walk.h"

#include "mem_dev.h"

namespace gc {
namespace {

using dev::gld;

// First node after k's subtree: the first later node whose id range starts at or after the end of
// k's (first ids never decrease along a pre-order numbering with contiguous id ranges), else n.
__global__ void __launch_bounds__(256) k_subtree_end(const int2* __restrict__ range, int32_t n,
                                                     int32_t* __restrict__ skip) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int2 r = gld(range + k);
  const int end = r.x + r.y;
  int lo = k + 1, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (gld(range + mid).x >= end) hi = mid;
    else lo = mid + 1;
  }
  skip[k] = lo;
}

struct WalkNode {
  int2 range;
  double com[3];
  double side;
  int skip;
};

// Node k's walk data; past the last node, a record that is never used (the walk stops there).
__device__ __forceinline__ WalkNode load_node(const WalkArgs& a, int k) {
  WalkNode w;
  if (k < a.n_nodes) {
    w.range = gld(a.range + k);
    w.com[0] = a.com[3 * (int64_t)k];
    w.com[1] = a.com[3 * (int64_t)k + 1];
    w.com[2] = a.com[3 * (int64_t)k + 2];
    w.side = a.side[k];
    w.skip = gld(a.skip + k);
  } else {
    w.range = make_int2(0, 0);
    w.com[0] = w.com[1] = w.com[2] = 0.0;
    w.side = 0.0;
    w.skip = k + 1;
  }
  return w;
}

template <bool FILL>
__global__ void __launch_bounds__(256) k_walk(WalkArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.n_buckets) return;
  const int leaf = gld(a.bucket_node + b);
  int2 br = make_int2(0, 0);
  bool ok = leaf >= 0 && leaf < a.n_nodes;
  if (ok) {
    br = gld(a.range + leaf);
    ok = br.x >= 0 && br.y >= 0 && br.x <= a.n_ids - br.y;
  }
  if (!ok) {  // an invalid bucket gets empty lists and is counted
    if (!FILL) {
      a.n_first[b] = 0;
      a.r_first[b] = 0;
      atomicAdd(a.bad, 1ull);
    }
    return;
  }
  double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
  double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
  for (int i = br.x; i < br.x + br.y; ++i) {
    const float4 p = gld(a.rec + i);
    const double v[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = v[d] < lo[d] ? v[d] : lo[d];
      hi[d] = v[d] > hi[d] ? v[d] : hi[d];
    }
  }
  int n_lim = 0, r_lim = 0, n_at = 0, r_at = 0;
  if (FILL) {  // the fill pass never writes past the bucket's counted share
    n_at = gld(a.n_first + b);
    n_lim = gld(a.n_first + b + 1) - n_at;
    r_at = gld(a.r_first + b);
    r_lim = gld(a.r_first + b + 1) - r_at;
    if (a.sn && n_lim <= kWalkCapNodes && r_lim <= kWalkCapRanges) return;  // copied from the count pass
  }
  int32_t* keep_n = (!FILL && a.sn) ? a.sn + (int64_t)kWalkCapNodes * b : nullptr;
  int2* keep_r = (!FILL && a.sn) ? a.sr + (int64_t)kWalkCapRanges * b : nullptr;
  int cn = 0, cr = 0;
  int kb0 = 0, kb1 = 0, kb2 = 0;  // node entries not yet kept (the last cn % 4)
  // both possible successors (k + 1 when k is opened, the end of k's subtree otherwise) are loaded at
  // the top of each step, so their latency overlaps the opening test of k
  WalkNode cur = load_node(a, 0);
  for (int k = 0; k < a.n_nodes;) {
    const int nxt = cur.skip;
    const WalkNode on_open = load_node(a, k + 1), on_skip = load_node(a, nxt);
    const int2 nr = cur.range;
    const bool disjoint = nr.x + nr.y <= br.x || br.x + br.y <= nr.x;
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double c = cur.com[d];
      double e = 0.0;
      if (c < lo[d]) e = __dsub_rn(lo[d], c);
      else if (c > hi[d]) e = __dsub_rn(c, hi[d]);
      s = __dadd_rn(s, __dmul_rn(e, e));
    }
    if (a.theta > 0.0 && disjoint && cur.side < __dmul_rn(a.theta, __dsqrt_rn(s))) {
      if (FILL && cn < n_lim) a.node_idx[n_at + cn] = k;
      if (!FILL && keep_n) {  // kept four at a time: one aligned 16-byte store per four entries
        const int slot = cn & 3;
        kb0 = slot == 0 ? k : kb0;
        kb1 = slot == 1 ? k : kb1;
        kb2 = slot == 2 ? k : kb2;
        if (slot == 3 && cn < kWalkCapNodes) *reinterpret_cast<int4*>(keep_n + (cn - 3)) = make_int4(kb0, kb1, kb2, k);
      }
      ++cn;
      k = nxt;
      cur = on_skip;
    } else if (nxt == k + 1) {
      if (FILL && cr < r_lim) {
        a.ranges[2 * (int64_t)(r_at + cr)] = nr.x;
        a.ranges[2 * (int64_t)(r_at + cr) + 1] = nr.y;
      }
      if (!FILL && keep_r && cr < kWalkCapRanges) keep_r[cr] = nr;
      ++cr;
      k = nxt;
      cur = on_skip;
    } else {
      k = k + 1;
      cur = on_open;
    }
  }
  if (!FILL && keep_n) {  // the last cn % 4 entries
    const int tail = cn & 3, at = cn - tail;
    if (tail > 0 && at < kWalkCapNodes) keep_n[at] = kb0;
    if (tail > 1 && at + 1 < kWalkCapNodes) keep_n[at + 1] = kb1;
    if (tail > 2 && at + 2 < kWalkCapNodes) keep_n[at + 2] = kb2;
  }
  if (!FILL) {
    a.n_first[b] = cn;
    a.r_first[b] = cr;
  }
}

// One wavefront per bucket: a bucket whose lists fit the count pass's room has them copied to its
// offsets (lanes over entries).
__global__ void __launch_bounds__(256) k_walk_copy(WalkArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= a.n_buckets) return;
  const int n_at = gld(a.n_first + b), n_cnt = gld(a.n_first + b + 1) - n_at;
  const int r_at = gld(a.r_first + b), r_cnt = gld(a.r_first + b + 1) - r_at;
  if (n_cnt > kWalkCapNodes || r_cnt > kWalkCapRanges) return;  // walked again by the fill pass
  const int32_t* src_n = a.sn + (int64_t)kWalkCapNodes * b;
  for (int i = lane; i < n_cnt; i += 64) a.node_idx[n_at + i] = gld(src_n + i);
  const int2* src_r = a.sr + (int64_t)kWalkCapRanges * b;
  for (int i = lane; i < r_cnt; i += 64) {
    const int2 v = gld(src_r + i);
    a.ranges[2 * (int64_t)(r_at + i)] = v.x;
    a.ranges[2 * (int64_t)(r_at + i) + 1] = v.y;
  }
}

// One workgroup of 1024 threads over tiles of 4096 entries of both arrays: each thread takes four
// consecutive entries, the threads' sums are scanned in LDS, and a carry runs from tile to tile.
__global__ void __launch_bounds__(1024) k_scan_counts(int32_t* __restrict__ a, int32_t* __restrict__ b, int32_t n,
                                                      long long* __restrict__ totals) {
  __shared__ long long sa[1024], sb[1024];
  const int t = threadIdx.x;
  long long carry_a = 0, carry_b = 0;
  for (int base = 0; base < n; base += 4096) {
    int va[4], vb[4];
    long long ta = 0, tb = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + 4 * t + q;
      va[q] = i < n ? a[i] : 0;
      vb[q] = i < n ? b[i] : 0;
      ta += va[q];
      tb += vb[q];
    }
    sa[t] = ta;
    sb[t] = tb;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const long long ua = t >= d ? sa[t - d] : 0, ub = t >= d ? sb[t - d] : 0;
      __syncthreads();
      sa[t] += ua;
      sb[t] += ub;
      __syncthreads();
    }
    long long pa = carry_a + sa[t] - ta, pb = carry_b + sb[t] - tb;  // exclusive prefix of the thread's entries
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + 4 * t + q;
      if (i < n) {
        a[i] = (int32_t)pa;
        b[i] = (int32_t)pb;
      }
      pa += va[q];
      pb += vb[q];
    }
    carry_a += sa[1023];
    carry_b += sb[1023];
    __syncthreads();  // sa / sb are rewritten by the next tile
  }
  if (t == 0) {
    a[n] = (int32_t)carry_a;
    b[n] = (int32_t)carry_b;
    totals[0] = carry_a;
    totals[1] = carry_b;
  }
}

}  // namespace

hipError_t launch_subtree_end(const int2* range, int32_t n_nodes, int32_t* skip, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_subtree_end, dim3((n_nodes + 255) / 256), dim3(256), 0, s, range, n_nodes, skip);
  return hipGetLastError();
}

hipError_t launch_walk(bool fill, const WalkArgs& a, hipStream_t s) {
  if (a.n_buckets <= 0) return hipSuccess;
  // one wavefront per workgroup: tens of thousands of buckets then spread over every CU
  const dim3 g((a.n_buckets + 63) / 64);
  if (fill) hipLaunchKernelGGL(k_walk<true>, g, dim3(64), 0, s, a);
  else hipLaunchKernelGGL(k_walk<false>, g, dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_walk_copy(const WalkArgs& a, hipStream_t s) {
  if (a.n_buckets <= 0 || !a.sn) return hipSuccess;
  hipLaunchKernelGGL(k_walk_copy, dim3((a.n_buckets + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scan_counts(int32_t* a, int32_t* b, int32_t n, long long* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, a, b, n, totals);
  return hipGetLastError();
}

}  // namespace gc
