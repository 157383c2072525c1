// Device code of the combined Barnes-Hut force pass (Sec. 3.1: many work
// requests in one launch; Sec. 4.1: a bucket's particles share one list of
// nodes and direct particles), shared by the per-batch kernel and the
// whole-step persistent kernel.
//
// Schedule: one workgroup of W wavefronts per task; the W waves split the
// task's node and direct lists.  A bucket holds few targets (about 10 on
// average for a Plummer sphere with buckets of 32), so within a wavefront the
// 64 lanes are split as (target i) x (source slice s): S = floor(64 / i_count)
// slices, lane = s * i_count + i.  Source records (direct particles, or node records) are
// staged by the wavefront into its private LDS tile with coalesced loads; the
// tile is padded with zero-mass entries to S * C records so every slice runs
// exactly C iterations with no per-iteration bounds test; a lane reads its
// slice's records from LDS (lanes of one slice read the same address: an LDS
// broadcast).  Node records of the next tile are prefetched into registers
// while the current tile is computed.  Each lane sums its slices in FP32 and
// adds that partial to an FP64 running sum once it holds 64 or more terms (a
// tile of more terms on its own), and at the end of the chunk; at the end the
// slices and then the waves of each target are reduced in FP64 through LDS in
// a fixed order and the target's float4 is written once.  No atomics: results
// are bitwise independent of task order and of the schedule.
//
// The inner loops are plain FP32 VALU code (v_sub / v_fma / v_mul) with the
// hardware reciprocal square root; pairwise forces are not a dense
// contraction, so no MFMA.
#pragma once

#include "gc_internal.h"
#include "mem_dev.h"

namespace gc {
namespace dev {

__device__ __forceinline__ void wave_sync() {
  // Lanes of one wavefront exchange data through wavefront-private LDS; the
  // LDS unit executes a wavefront's instructions in order, so only compiler
  // reordering must be prevented here.
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
  const int lane = threadIdx.x & 63;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  *total = __shfl(inc, 63, 64);
  return inc - v;
}

// Sum over a tile of C pair/monopole records per slice: p = records of this lane's slice.
__device__ __forceinline__ void tile_pairs(const float4* __restrict__ p, int C, float xi, float yi, float zi,
                                           float eps2, float& ax, float& ay, float& az) {
  int k = 0;
  for (; k + 4 <= C; k += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float4 j = p[k + u];
      float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
      float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
      float ri = __builtin_amdgcn_rsqf(r2);
      float mr = j.w * ri;
      float ri2 = ri * ri;
      float sc = mr * ri2;
      ax = __builtin_fmaf(dx, sc, ax);
      ay = __builtin_fmaf(dy, sc, ay);
      az = __builtin_fmaf(dz, sc, az);
    }
  }
  for (; k < C; ++k) {
    float4 j = p[k];
    float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
    float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    float ri = __builtin_amdgcn_rsqf(r2);
    float mr = j.w * ri;
    float ri2 = ri * ri;
    float sc = mr * ri2;
    ax = __builtin_fmaf(dx, sc, ax);
    ay = __builtin_fmaf(dy, sc, ay);
    az = __builtin_fmaf(dz, sc, az);
  }
}

// Quadrupole node records in LDS: (com, M), (3Sxx, 3Syy, 3Szz, 3Sxy), (3Sxz, 3Syz, 1.5 T, 0).
__device__ __forceinline__ void tile_quads(const float4* __restrict__ p, int C, float xi, float yi, float zi,
                                           float eps2, float& ax, float& ay, float& az) {
#pragma unroll 2
  for (int k = 0; k < C; ++k) {
    float4 a = p[3 * k], b = p[3 * k + 1], c = p[3 * k + 2];
    float dx = xi - a.x, dy = yi - a.y, dz = zi - a.z;
    float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    float ri = __builtin_amdgcn_rsqf(r2);
    float q = ri * ri;
    float r3 = ri * q;
    float r5 = r3 * q;
    // S' d with S' = 3 S
    float sx = __builtin_fmaf(c.x, dz, __builtin_fmaf(b.w, dy, b.x * dx));
    float sy = __builtin_fmaf(c.y, dz, __builtin_fmaf(b.y, dy, b.w * dx));
    float sz = __builtin_fmaf(b.z, dz, __builtin_fmaf(c.y, dy, c.x * dx));
    float dsd = __builtin_fmaf(dz, sz, __builtin_fmaf(dy, sy, dx * sx));  // 3 d.S.d
    // coefficient of d: -M r^-3 + 1.5 T r^-5 - 7.5 (d.S.d) r^-7 = r^-3 (-M + q (1.5 T - 2.5 q dsd))
    float u = __builtin_fmaf(dsd, q * -2.5f, c.z);
    float v = __builtin_fmaf(q, u, -a.w);
    float cf = r3 * v;
    ax = __builtin_fmaf(r5, sx, __builtin_fmaf(cf, dx, ax));
    ay = __builtin_fmaf(r5, sy, __builtin_fmaf(cf, dy, ay));
    az = __builtin_fmaf(r5, sz, __builtin_fmaf(cf, dz, az));
  }
}

// The same tiles with the potential: ph accumulates m r^-1 (pair, monopole) and, for a quadrupole
// node, M r^-1 + 1/2 (d.S'.d) r^-5 - (1.5 T / 3) r^-3 with S' = 3 S, i.e. M/r + 3/2 d.S.d/r^5 - T/(2r^3);
// the caller scales by -G.
__device__ __forceinline__ void tile_pairs_pot(const float4* __restrict__ p, int C, float xi, float yi, float zi,
                                               float eps2, float& ax, float& ay, float& az, float& ph) {
  for (int k = 0; k < C; ++k) {
    float4 j = p[k];
    float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
    float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    float ri = __builtin_amdgcn_rsqf(r2);
    float mr = j.w * ri;
    float ri2 = ri * ri;
    float sc = mr * ri2;
    ax = __builtin_fmaf(dx, sc, ax);
    ay = __builtin_fmaf(dy, sc, ay);
    az = __builtin_fmaf(dz, sc, az);
    ph += mr;
  }
}

__device__ __forceinline__ void tile_quads_pot(const float4* __restrict__ p, int C, float xi, float yi, float zi,
                                               float eps2, float& ax, float& ay, float& az, float& ph) {
  for (int k = 0; k < C; ++k) {
    float4 a = p[3 * k], b = p[3 * k + 1], c = p[3 * k + 2];
    float dx = xi - a.x, dy = yi - a.y, dz = zi - a.z;
    float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    float ri = __builtin_amdgcn_rsqf(r2);
    float q = ri * ri;
    float r3 = ri * q;
    float r5 = r3 * q;
    float sx = __builtin_fmaf(c.x, dz, __builtin_fmaf(b.w, dy, b.x * dx));
    float sy = __builtin_fmaf(c.y, dz, __builtin_fmaf(b.y, dy, b.w * dx));
    float sz = __builtin_fmaf(b.z, dz, __builtin_fmaf(c.y, dy, c.x * dx));
    float dsd = __builtin_fmaf(dz, sz, __builtin_fmaf(dy, sy, dx * sx));
    float u = __builtin_fmaf(dsd, q * -2.5f, c.z);
    float v = __builtin_fmaf(q, u, -a.w);
    float cf = r3 * v;
    ax = __builtin_fmaf(r5, sx, __builtin_fmaf(cf, dx, ax));
    ay = __builtin_fmaf(r5, sy, __builtin_fmaf(cf, dy, ay));
    az = __builtin_fmaf(r5, sz, __builtin_fmaf(cf, dz, az));
    ph += __builtin_fmaf(0.5f * dsd, r5, __builtin_fmaf(a.w, ri, c.z * (-1.f / 3.f) * r3));
  }
}

// One pair or monopole term and one quadrupole term for one target (the same arithmetic as the
// loops above), used by the two-targets-per-lane tiles below.
__device__ __forceinline__ void pair_term(const float4 j, float xi, float yi, float zi, float eps2, float& ax,
                                          float& ay, float& az) {
  float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
  float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
  float ri = __builtin_amdgcn_rsqf(r2);
  float mr = j.w * ri;
  float ri2 = ri * ri;
  float sc = mr * ri2;
  ax = __builtin_fmaf(dx, sc, ax);
  ay = __builtin_fmaf(dy, sc, ay);
  az = __builtin_fmaf(dz, sc, az);
}

__device__ __forceinline__ void quad_term(const float4 a, const float4 b, const float4 c, float xi, float yi, float zi,
                                          float eps2, float& ax, float& ay, float& az) {
  float dx = xi - a.x, dy = yi - a.y, dz = zi - a.z;
  float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
  float ri = __builtin_amdgcn_rsqf(r2);
  float q = ri * ri;
  float r3 = ri * q;
  float r5 = r3 * q;
  float sx = __builtin_fmaf(c.x, dz, __builtin_fmaf(b.w, dy, b.x * dx));
  float sy = __builtin_fmaf(c.y, dz, __builtin_fmaf(b.y, dy, b.w * dx));
  float sz = __builtin_fmaf(b.z, dz, __builtin_fmaf(c.y, dy, c.x * dx));
  float dsd = __builtin_fmaf(dz, sz, __builtin_fmaf(dy, sy, dx * sx));
  float u = __builtin_fmaf(dsd, q * -2.5f, c.z);
  float v = __builtin_fmaf(q, u, -a.w);
  float cf = r3 * v;
  ax = __builtin_fmaf(r5, sx, __builtin_fmaf(cf, dx, ax));
  ay = __builtin_fmaf(r5, sy, __builtin_fmaf(cf, dy, ay));
  az = __builtin_fmaf(r5, sz, __builtin_fmaf(cf, dz, az));
}

// Terms per lane summed in FP32 before they are added into the FP64 sums of a target chunk.
constexpr int kFlushTerms = 64;

// Two targets per lane: each record read from LDS serves both (half the LDS reads per interaction,
// two independent dependency chains per lane).
struct Acc2 {
  float ax, ay, az, bx, by, bz;
};

__device__ __forceinline__ void tile_pairs2(const float4* __restrict__ p, int C, const float3 A, const float3 B,
                                            float eps2, Acc2& r) {
  int k = 0;
  for (; k + 2 <= C; k += 2) {
    const float4 j0 = p[k], j1 = p[k + 1];
    pair_term(j0, A.x, A.y, A.z, eps2, r.ax, r.ay, r.az);
    pair_term(j0, B.x, B.y, B.z, eps2, r.bx, r.by, r.bz);
    pair_term(j1, A.x, A.y, A.z, eps2, r.ax, r.ay, r.az);
    pair_term(j1, B.x, B.y, B.z, eps2, r.bx, r.by, r.bz);
  }
  if (k < C) {
    const float4 j0 = p[k];
    pair_term(j0, A.x, A.y, A.z, eps2, r.ax, r.ay, r.az);
    pair_term(j0, B.x, B.y, B.z, eps2, r.bx, r.by, r.bz);
  }
}

__device__ __forceinline__ void tile_quads2(const float4* __restrict__ p, int C, const float3 A, const float3 B,
                                            float eps2, Acc2& r) {
  for (int k = 0; k < C; ++k) {
    const float4 a = p[3 * k], b = p[3 * k + 1], c = p[3 * k + 2];
    quad_term(a, b, c, A.x, A.y, A.z, eps2, r.ax, r.ay, r.az);
    quad_term(a, b, c, B.x, B.y, B.z, eps2, r.bx, r.by, r.bz);
  }
}

// Node record for LDS: monopole (com, M); quadrupole adds (3 Sxx, 3 Syy, 3 Szz, 3 Sxy), (3 Sxz, 3 Syz, 1.5 T, 0).
template <int ORDER>
struct NodeRegs {
  float4 v0, v1, v2;
};

// The node table as a raw buffer (three records, 48 bytes, a node).  A load past its end returns
// zeros, so a lane without a node (index < 0) loads a zero record with no branch and no zeroing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t node_rsrc(const float4* nodes, int32_t n_nodes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float4*>(nodes), (short)0, n_nodes * 48, 0x00020000);
}

__device__ __forceinline__ float4 u4f(const __attribute__((ext_vector_type(4))) unsigned v) {
  return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

template <int ORDER>
__device__ __forceinline__ NodeRegs<ORDER> load_node(__amdgpu_buffer_rsrc_t nodes, int idx) {
  NodeRegs<ORDER> r;
  // (node indices are below 2^24, checked on the host: a full-rate 24-bit multiply)
  const int off = idx >= 0 ? (int)__umul24((unsigned)idx, 48u) : 0x7ffffff0;  // past the end of any node table
  r.v0 = u4f(__builtin_amdgcn_raw_buffer_load_b128(nodes, off, 0, 0));
  if (ORDER == 2) {
    r.v1 = u4f(__builtin_amdgcn_raw_buffer_load_b128(nodes, off + 16, 0, 0));
    // the third record's fourth word is padding: three words
    const __attribute__((ext_vector_type(3))) unsigned c = __builtin_amdgcn_raw_buffer_load_b96(nodes, off + 32, 0, 0);
    r.v2 = make_float4(__uint_as_float(c[0]), __uint_as_float(c[1]), __uint_as_float(c[2]), 0.f);
  } else {
    r.v1 = r.v2 = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  return r;
}

template <int ORDER>
__device__ __forceinline__ void store_node(float4* L, int e, const NodeRegs<ORDER>& r) {
  if (ORDER == 1) {
    L[e] = r.v0;
  } else {
    L[3 * e] = r.v0;
    L[3 * e + 1] = make_float4(3.f * r.v1.x, 3.f * r.v1.y, 3.f * r.v1.z, 3.f * r.v1.w);
    L[3 * e + 2] = make_float4(3.f * r.v2.x, 3.f * r.v2.y, 1.5f * r.v2.z, 0.f);
  }
}

// The first node tile of a task for the calling wavefront (nodes w, w + W, ... of the task's list):
// the records in registers, one node per lane, and the index of the node 64 entries on.
template <int ORDER>
struct NodePrefetch {
  NodeRegs<ORDER> cur;
  int idx_next;
};

template <int ORDER>
__device__ __forceinline__ void node_prefetch(__amdgpu_buffer_rsrc_t nodes, const int* __restrict__ node_idx,
                                              int n_first, int n_count, NodePrefetch<ORDER>& pf) {
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const int nw = n_count > wid ? (n_count - wid + W - 1) / W : 0;
  const int* nl = node_idx + n_first + wid;
  const int lw = lane * W;
  pf.idx_next = (64 < nw && 64 + lane < nw) ? gld(nl + (lw + 64 * W)) : -1;
  pf.cur = load_node<ORDER>(nodes, lane < nw ? gld(nl + lw) : -1);
}

// Records of LDS per wavefront for a direct tile of `tile` records: the larger of a direct tile and
// a quadrupole node tile (3 records per node), plus 96 records of reduction scratch.  A tile holds a
// multiple of the slice count S and is padded to S * ceil(count / S) records, which never exceeds
// that multiple, so the padding needs no room of its own.  (The larger area also holds the 6 x 64
// FP64 sums of the two-targets reduction: 192 records.)
__host__ __device__ __forceinline__ int grav_rec_cap(int tile) {
  return tile > 3 * kNodeTile ? tile : 3 * kNodeTile;
}
// With the potential (POT) the reduction scratch holds four sums per lane: 128 records.
__host__ __device__ __forceinline__ int grav_lds_per_wave(int tile, bool pot = false) {
  return grav_rec_cap(tile) + (pot ? 128 : 96);
}

// Two targets per lane fill more of the wavefront than one for a task of n targets (n = i_count,
// at most 64 counted) when floor(64 / ceil(n / 2)) slices of lane pairs hold more than twice
// floor(64 / n) slices of single lanes (n = 6, 13, 14, 17, 18, 22, 23, 24 and 33 to 42); otherwise
// one target per lane is at least as full and reads no duplicate target.
__host__ __device__ __forceinline__ bool two_fills_more(int n) {
  n = n < 64 ? n : 64;
  return n > 0 && 64 / ((n + 1) >> 1) > 2 * (64 / n);
}

// A task as the force code reads it: the submitted fields and the first target's position in the
// record array (its packed position, or i_begin when records are read in place).
struct TaskDesc {
  int32_t i_begin, i_count, j_first, j_nranges, n_first, n_count, ibeg;
};

// One task on one workgroup of W = blockDim.x / 64 wavefronts.  Wave w takes the task's nodes
// w, w + W, ... and the w-th of W contiguous, nearly equal shares of its direct records (address
// lists: windows w, w + W, ...), so W waves share one task's lists.  Within a wave the lanes are (lane-target j) x (slice s): with
// two targets per lane (TPL 2) each lane carries targets j and j + h (h = ceil(i_count / 2)),
// otherwise (TPL 1) target j (h = i_count); S = floor(64 / h) slices.  The per-target sums are reduced across slices within each
// wave and then across the W waves, in a fixed order.  `smem` is the block's dynamic LDS of
// W * grav_lds_per_wave(tile) records; the call starts and ends with every wave of the block
// converged (it contains block barriers).  pf holds the task's first node tile when `have_pf`
// (loaded ahead by the caller), else it is loaded here.  ready() is called by every thread once the
// first node tile's loads are out and before any record is read (the records may still be being
// written).  In the last target chunk next(0) and, after a block barrier, next(1) are called by
// every thread before the cross-wave sum; next(1) may load the following task's first node tile
// into pf.  The last barrier is the caller's: it must sync the block before the LDS is reused.
// POT (one target per lane, records in position space): acc.w also receives the potential of the
// task's terms, -G times the sum above, without the target's own direct term (a target found in its
// task's direct ranges has contributed m r^-1 at r = eps, which is taken out again).
template <int ORDER, bool LISTS, int TPL, bool POT = false, class Ready, class Next>
__device__ __forceinline__ void grav_task_body(const GravArgs& a, const int t, const TaskDesc& tk,
                                          float4* __restrict__ smem, NodePrefetch<ORDER>& pf, bool have_pf,
                                          Ready&& ready, Next&& next) {
  static_assert(TPL == 1 || TPL == 2, "one or two targets per lane");
  static_assert(!POT || (TPL == 1 && !LISTS), "the potential runs one target per lane in position space");
  constexpr int NC = POT ? 4 : 3;  // sums per target
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int W = blockDim.x >> 6;
  const int tile = a.tile;
  const int rec_cap = grav_rec_cap(tile);
  const int per_wave = grav_lds_per_wave(tile, POT);
  float4* L = smem + wid * per_wave;
  double* red = reinterpret_cast<double*>(L + rec_cap);
  // the range tables of the direct phase share the reduction scratch (live at different times)
  int* RO = reinterpret_cast<int*>(red);  // range start offsets within the group (64)
  int* RB = RO + 64;                      // range begins (64)
  const int ic = tk.i_count;
  // this wave's nodes; the first tile does not depend on the records, so its loads go out first
  const int nw = tk.n_count > wid ? (tk.n_count - wid + W - 1) / W : 0;
  const int* nl = a.node_idx + tk.n_first + wid;
  const int lw = lane * W;  // nl[lw + e * W] is this lane's entry e + lane
  const __amdgpu_buffer_rsrc_t nodes = node_rsrc(a.nodes, a.n_nodes);
  if (!have_pf) node_prefetch<ORDER>(nodes, a.node_idx, tk.n_first, tk.n_count, pf);
  ready();
  for (int i0 = 0; i0 < ic; i0 += 64) {
    if (i0 > 0) node_prefetch<ORDER>(nodes, a.node_idx, tk.n_first, tk.n_count, pf);
    const bool last = i0 + 64 >= ic;
    const int icc = ic - i0 < 64 ? ic - i0 : 64;
    constexpr bool two = TPL == 2;
    const int h = two ? (icc + 1) >> 1 : icc;
    const int S = uniform(64 / h);
    // lane / h and lane % h by a multiply: floor(lane * ceil(2^16 / h) / 2^16) = floor(lane / h) for
    // lane < 64 and h <= 64 (the rounding error stays below 1 / h)
    const uint32_t mh = (uint32_t)uniform((65536 + h - 1) / h);
    const int sl = (int)(((uint32_t)lane * mh) >> 16);
    const int il = lane - sl * h;
    const int sl3 = 3 * sl;
    const bool active = sl < S;
    // tiles hold a multiple of S records, so that only a share's last tile is padded
    const int NT = uniform(S * (kNodeTile / S));  // nodes per node tile
    const int DT = uniform(S * (tile / S));       // records per direct tile
    const int ib = il + h < icc ? il + h : il;  // two: second target (a copy of the first if absent)
    float3 A = make_float3(0.f, 0.f, 0.f), B = A;
    if (active) {
      const int pb = LISTS ? 0 : tk.ibeg + i0;
      const float4 r = gld(a.rec + (LISTS ? gld(a.ilist + gld(a.ioff + t) + i0 + il) : pb + il));
      A = make_float3(r.x, r.y, r.z);
      if (two) {
        const float4 q = gld(a.rec + (LISTS ? gld(a.ilist + gld(a.ioff + t) + i0 + ib) : pb + ib));
        B = make_float3(q.x, q.y, q.z);
      }
    }
    double Ax = 0.0, Ay = 0.0, Az = 0.0, Bx = 0.0, By = 0.0, Bz = 0.0, Ap = 0.0;
    // FP32 sums carried across tiles and added into the FP64 ones once they hold kFlushTerms terms
    // or more per lane (a run stays below kFlushTerms + C terms, and a tile of C >= kFlushTerms
    // terms is added on its own), and before the reduction
    Acc2 f{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float fp = 0.f;
    int fcnt = 0;  // uniform
    auto flush = [&]() {
      Ax += f.ax; Ay += f.ay; Az += f.az;
      if (two) {
        Bx += f.bx; By += f.by; Bz += f.bz;
      }
      if (POT) Ap += fp;
      f = Acc2{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      fp = 0.f;
      fcnt = 0;
    };
    // one tile of C records per slice starting at L + rec_stride * sl * C: accumulate it
    auto tile_sum = [&](int C, bool quads) {
      if (active) {
        if (two) {
          if (quads) tile_quads2(L + __mul24(sl3, C), C, A, B, a.eps2, f);
          else tile_pairs2(L + __mul24(sl, C), C, A, B, a.eps2, f);
        } else if (POT) {
          if (quads) tile_quads_pot(L + __mul24(sl3, C), C, A.x, A.y, A.z, a.eps2, f.ax, f.ay, f.az, fp);
          else tile_pairs_pot(L + __mul24(sl, C), C, A.x, A.y, A.z, a.eps2, f.ax, f.ay, f.az, fp);
        } else {
          if (quads) tile_quads(L + __mul24(sl3, C), C, A.x, A.y, A.z, a.eps2, f.ax, f.ay, f.az);
          else tile_pairs(L + __mul24(sl, C), C, A.x, A.y, A.z, a.eps2, f.ax, f.ay, f.az);
        }
      }
      fcnt += C;
      if (fcnt >= kFlushTerms) flush();
    };

    // ---- node terms: this wave's nodes are list entries w, w + W, ...
    {
      // the prefetched first tile holds nodes 0..63 and the index of node 64 + lane; with NT < 64
      // its lanes >= NT are left out (zero records) and the next tile starts at node NT.  Every
      // tile's lanes past its last node then hold zero records: the padding of the tile
      if (NT < kNodeTile) {
        pf.idx_next = (lane < NT && NT + lane < nw) ? gld(nl + (lw + NT * W)) : -1;
        if (lane >= NT) pf.cur = load_node<ORDER>(nodes, -1);
      }
      for (int nb = 0; nb < nw; nb += NT) {
        const int cnt = nw - nb < NT ? nw - nb : NT;
        const int C = uniform((cnt + S - 1) / S);
        store_node<ORDER>(L, lane, pf.cur);
        // prefetch the next tile's records and the index of the one after
        if (nb + NT < nw) {
          pf.cur = load_node<ORDER>(nodes, pf.idx_next);
          const int e2 = nb + 2 * NT + lane;
          pf.idx_next = (lane < NT && e2 < nw) ? gld(nl + (lw + (nb + 2 * NT) * W)) : -1;
        }
        wave_sync();
        // monopole: a = -M d / r^3 with d = x_i - com, the same as a pair term from a source at com
        tile_sum(C, ORDER == 2);
        wave_sync();
      }
    }

    // ---- direct terms
    if (LISTS) {
      const int jb = gld(a.joff + t), jn = gld(a.joff + t + 1) - jb;
      for (int ws = wid * DT; ws < jn; ws += W * DT) {
        const int cnt = jn - ws < DT ? jn - ws : DT;
        const int C = uniform((cnt + S - 1) / S);
        const int padded = S * C;
        for (int e = lane; e < padded; e += 64) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (e < cnt) v = gld(a.rec + gld(a.jlist + jb + ws + e));
          L[e] = v;
        }
        wave_sync();
        tile_sum(C, false);
        wave_sync();
      }
    } else {
      // the task's ranges in groups of 64, each flattened by a wave scan; wave w takes the w-th of
      // W contiguous, nearly equal shares of every group's records, and each lane copies one flat
      // position, finding its range by binary search over the offsets kept in LDS
      const int2* rl = a.ranges + tk.j_first;
      for (int rg = 0; rg < tk.j_nranges; rg += 64) {
        const int nr = tk.j_nranges - rg < 64 ? tk.j_nranges - rg : 64;
        int2 g = make_int2(0, 0);
        if (lane < nr) g = gld(rl + rg + lane);
        int total;
        const int o = wave_excl_scan(g.y, &total);
        total = uniform(total);
        RO[lane] = lane < nr ? o : 0x7fffffff;
        RB[lane] = g.x;
        wave_sync();
        // share boundaries rounded down to multiples of S (the last share ends at the total)
        // (32-bit: a task's direct records stay below 2^28)
        const int lo = uniform((int)((uint32_t)total * (uint32_t)wid / (uint32_t)W / (uint32_t)S) * S);
        const int hi = wid + 1 == W ? total
                                    : uniform((int)((uint32_t)total * (uint32_t)(wid + 1) / (uint32_t)W / (uint32_t)S) * S);
        for (int ws = lo; ws < hi; ws += DT) {
          const int cnt = hi - ws < DT ? hi - ws : DT;
          const int C = uniform((cnt + S - 1) / S);
          const int padded = S * C;
          for (int e = lane; e < padded; e += 64) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < cnt) {
              const int f = ws + e;
              int lo = 0, hi = nr - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (RO[mid] <= f) lo = mid;
                else hi = mid - 1;
              }
              v = gld(a.rec + RB[lo] + (f - RO[lo]));
            }
            L[e] = v;
          }
          wave_sync();
          tile_sum(C, false);
          wave_sync();
        }
      }
    }

    // ---- reduce: slices within the wave, then the W waves, in a fixed order
    flush();
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
    if (two) {
      // 6 sums per lane: the tile area is free now
      double* R2 = reinterpret_cast<double*>(L);
      R2[6 * lane] = Ax; R2[6 * lane + 1] = Ay; R2[6 * lane + 2] = Az;
      R2[6 * lane + 3] = Bx; R2[6 * lane + 4] = By; R2[6 * lane + 5] = Bz;
      wave_sync();
      if (lane < icc) {
        const int j = lane < h ? lane : lane - h, off = lane < h ? 0 : 3;
        for (int s = 0; s < S; ++s) {
          const double* q = R2 + 6 * (s * h + j) + off;
          sx += q[0]; sy += q[1]; sz += q[2];
        }
      }
    } else {
      red[NC * lane] = Ax;
      red[NC * lane + 1] = Ay;
      red[NC * lane + 2] = Az;
      if (POT) red[NC * lane + 3] = Ap;
      wave_sync();
      if (lane < icc) {
        for (int s = 0; s < S; ++s) {
          const double* q = red + NC * (s * icc + lane);
          sx += q[0]; sy += q[1]; sz += q[2];
          if (POT) sp += q[3];
        }
      }
    }
    wave_sync();
    if (lane < icc) {
      red[NC * lane] = sx;
      red[NC * lane + 1] = sy;
      red[NC * lane + 2] = sz;
      if (POT) red[NC * lane + 3] = sp;
    }
    if (last) next(0);
    __syncthreads();
    if (last) next(1);
    if (wid == 0 && lane < icc) {
      double tx = 0.0, ty = 0.0, tz = 0.0, tp = 0.0;
      for (int w = 0; w < W; ++w) {
        const double* q = reinterpret_cast<const double*>(smem + w * per_wave + rec_cap) + NC * lane;
        tx += q[0]; ty += q[1]; tz += q[2];
        if (POT) tp += q[3];
      }
      float phi = 0.f;
      if (POT) {
        // the target's own direct term, if its position lies in one of the task's ranges
        const int pos = tk.ibeg + i0 + lane;
        bool self = false;
        for (int r = 0; r < tk.j_nranges; ++r) {
          const int2 g = gld(a.ranges + tk.j_first + r);
          self = self || (pos >= g.x && pos < g.x + g.y);
        }
        if (self) tp -= (double)(gld(a.rec + pos).w * __builtin_amdgcn_rsqf(a.eps2));
        phi = (float)(-a.G * tp);
      }
      gst(a.acc + tk.i_begin + i0 + lane, make_float4((float)(a.G * tx), (float)(a.G * ty), (float)(a.G * tz), phi));
    }
    if (!last) __syncthreads();
  }
}

// A task in targets-per-lane mode TPL: 1 or 2 as above; 3 chooses per task, two where they fill more
// lanes (two_fills_more), so that each form's registers are live only in its own branch.
template <int ORDER, bool LISTS, int TPL, bool POT = false, class Ready, class Next>
__device__ __forceinline__ void grav_task(const GravArgs& a, const int t, const TaskDesc& tk,
                                          float4* __restrict__ smem, NodePrefetch<ORDER>& pf, bool have_pf,
                                          Ready&& ready, Next&& next) {
  if constexpr (TPL == 3) {
    if (two_fills_more(tk.i_count))
      grav_task_body<ORDER, LISTS, 2, POT>(a, t, tk, smem, pf, have_pf, ready, next);
    else
      grav_task_body<ORDER, LISTS, 1, POT>(a, t, tk, smem, pf, have_pf, ready, next);
  } else {
    grav_task_body<ORDER, LISTS, TPL, POT>(a, t, tk, smem, pf, have_pf, ready, next);
  }
}

}  // namespace dev
}  // namespace gc
