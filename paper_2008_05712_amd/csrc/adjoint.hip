// Adjoint (vector-Jacobian product) of the combined force pass for
// L = sum_i cot_i . a_i, recomputing every pair term (nothing is stored by
// the forward pass).
//
// Gravity (direct + monopole nodes).  With u = x_j - x_i, s^2 = |u|^2 + eps^2:
//   w = G m_j [g_i / s^3 - 3 (g_i . u) u / s^5];  dL/dx_j += w, dL/dx_i -= w,
//   dL/dm_j += G (g_i . u) / s^3   (the i = j term is skipped)
// and for a node with d = x_i - com, r^2 = |d|^2 + eps^2:
//   v = -G M [g_i / r^3 - 3 (g_i . d) d / r^5];  dL/dx_i += v, dL/dcom -= v,
//   dL/dM += -G (g_i . d) / r^3.
// and with quadrupole nodes (S the raw second moment, T = tr S, q = d.S.d) also
//   d(g.a_q)/dd = G [3 S g / r^5 - 15 (g.Sd) d / r^7 - 15 (g.d) S d / r^7 - 15/2 q g / r^7
//                    + 105/2 q (g.d) d / r^9 + 3/2 T g / r^5 - 15/2 T (g.d) d / r^7]  (to x_i, minus to com),
//   H = sym(dL/dS) = G [3/2 (g d^T + d g^T) / r^5 - 15/2 (g.d) d d^T / r^7 + 3/2 (g.d) I / r^5].
// Node gradients reach member particles through com = sum m_k x_k / M, M = sum m_k and
// S = sum m_k e_k e_k^T (e_k = x_k - com):  dL/dx_k += (m_k / M) dL/dcom + 2 m_k H e_k,
// dL/dm_k += dL/dM + e_k . dL/dcom / M + e_k . H e_k.
//
// Schedule: one workgroup of 4 wavefronts per task, splitting its sources;
// lanes are sources (nodes, then direct particles), the loop runs over
// blocks of 8 targets (6 with quadrupole nodes) held in registers
// (LDS broadcast), so each lane accumulates its source's gradient across
// the block and each target's gradient is reduced across the wavefront once
// per block (then added with an FP32 atomic: order-dependent rounding).  A
// source's gradient from one task is kept in a record of its own, one per
// visit (entry of a node list, flat direct position): the lane that owns the
// visit adds each block's part to it, so nothing contends.  The records are
// then gathered through per-node and per-particle visit indices and summed in
// a fixed order; the node sums reach the member particles through the chain.
//
// Lennard-Jones: h_i = g_i / m_i, dh = h_i - h_j, p = dh . d, f' = df/d(r^2):
//   dL/dx_i += f dh + 2 f' p d, dL/dx_j -= the same,
//   dL/deps_ij = p f / eps_ij,  dL/dsigma_ij = p * 24 eps (24 s^11 r^-14 - 6 s^5 r^-8),
//   chained to the per-type parameters through Lorentz-Berthelot mixing;
//   dL/dm_i = -g_i . F_i / m_i^2 with the forces F recomputed here.
// When the batch's target ranges are equal or disjoint, the gather form runs: as the forward gather
// form, one wavefront per target cell over every task touching it from either side.  The pair term
// is the same from both sides: with e the separation seen from the target and h_t, h_s the target's
// and the source's g / m, the target takes f (h_t - h_s) + 2 f' ((h_t - h_s) . e) e, and each side
// adds half of the pair's parameter derivatives.
#include "gc_internal.h"
#include "grav_dev.h"
#include "mem_dev.h"

namespace gc {
namespace {

using dev::gld;
using dev::gst;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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

// One workgroup of W wavefronts per task (1 to 4): wave w takes the task's nodes w, w + W, ... and
// the flat direct positions of every W-th group of 64; source gradients go to the visits' records
// and target gradients are added with atomics, so the waves need no reduction among themselves.
template <bool PACKED, int ORDER>
__global__ void __launch_bounds__(256) k_grav_adj(GravAdjArgs A) {
  // targets per register block: six with quadrupole nodes keep the kernel at three wavefronts per SIMD
  constexpr int kTB = ORDER == 2 ? 6 : 8;
  const GravArgs& a = A.f;
  __shared__ float4 tpos[4][kTB], tcot[4][kTB];
  __shared__ int ro[4][64], rb[4][64];
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int W = uniform(blockDim.x >> 6);  // 1 to 4
  const int t = uniform(blockIdx.x);
  if (t >= a.n_tasks) return;
  const gc_task tk = a.tasks[t];
  const int ic = tk.i_count;
  const int ibase = PACKED ? a.ibeg[t] : tk.i_begin;
  const float G = a.G, eps2 = a.eps2;
  for (int tb0 = 0; tb0 < ic; tb0 += kTB) {
    const int tb = uniform(ic - tb0 < kTB ? ic - tb0 : kTB);
    if (lane < kTB) {
      float4 p = make_float4(0.f, 0.f, 0.f, 0.f), g = p;
      if (lane < tb) {
        p = a.rec[ibase + tb0 + lane];
        g = A.cot[tk.i_begin + tb0 + lane];
      }
      tpos[wid][lane] = p;
      tcot[wid][lane] = g;
    }
    wave_sync();
    float xt[kTB], yt[kTB], zt[kTB], gx[kTB], gy[kTB], gz[kTB];
    int idt[kTB];
    float tgx[kTB], tgy[kTB], tgz[kTB];
#pragma unroll
    for (int k = 0; k < kTB; ++k) {
      float4 p = tpos[wid][k], g = tcot[wid][k];
      xt[k] = p.x; yt[k] = p.y; zt[k] = p.z;
      gx[k] = g.x; gy[k] = g.y; gz[k] = g.z;
      idt[k] = k < tb ? tk.i_begin + tb0 + k : -1;
      tgx[k] = tgy[k] = tgz[k] = 0.f;
    }
    // ---- nodes: lane = node
    for (int nb = wid * 64; nb < tk.n_count; nb += W * 64) {
      const int e = nb + lane;
      const bool valid = e < tk.n_count;
      int nd = -1;
      float4 c = make_float4(0.f, 0.f, 0.f, 0.f), s1 = c, s2 = c;
      if (valid) {
        nd = a.node_idx[tk.n_first + e];
        c = a.nodes[3 * nd];
        if (ORDER == 2) {
          s1 = a.nodes[3 * nd + 1];  // Sxx Syy Szz Sxy
          s2 = a.nodes[3 * nd + 2];  // Sxz Syz T
        }
      }
      const float GM = G * c.w;
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gM = 0.f;
      float hxx = 0.f, hyy = 0.f, hzz = 0.f, hxy = 0.f, hxz = 0.f, hyz = 0.f;  // sym(dL/dS) / G
#pragma unroll
      for (int k = 0; k < kTB; ++k) {
        if (k >= tb) break;  // (uniform) targets past the block's last do no work
        float dx = xt[k] - c.x, dy = yt[k] - c.y, dz = zt[k] - c.z;
        float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
        float ri = __builtin_amdgcn_rsqf(r2);
        float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
        float gd = __builtin_fmaf(gz[k], dz, __builtin_fmaf(gy[k], dy, gx[k] * dx));
        float c1 = -GM * ri3;
        float c2 = 3.f * GM * gd * ri5;
        float vx = __builtin_fmaf(c1, gx[k], c2 * dx);
        float vy = __builtin_fmaf(c1, gy[k], c2 * dy);
        float vz = __builtin_fmaf(c1, gz[k], c2 * dz);
        if (ORDER == 2) {
          // d(g.a_q)/dd = G [3 (S g / r^5 - 5 (g.Sd) d / r^7) - 15/2 (2 (g.d) S d / r^7 + q g / r^7
          //                  - 7 q (g.d) d / r^9) + 3/2 T (g / r^5 - 5 (g.d) d / r^7)],  q = d.S.d
          const float ri7 = ri5 * ri2, ri9 = ri7 * ri2;
          const float sdx = s1.x * dx + s1.w * dy + s2.x * dz;
          const float sdy = s1.w * dx + s1.y * dy + s2.y * dz;
          const float sdz = s2.x * dx + s2.y * dy + s1.z * dz;
          const float sgx = s1.x * gx[k] + s1.w * gy[k] + s2.x * gz[k];
          const float sgy = s1.w * gx[k] + s1.y * gy[k] + s2.y * gz[k];
          const float sgz = s2.x * gx[k] + s2.y * gy[k] + s1.z * gz[k];
          const float q = dx * sdx + dy * sdy + dz * sdz;
          const float gsd = gx[k] * sdx + gy[k] * sdy + gz[k] * sdz;
          const float T = s2.z;
          const float kS = 3.f * ri5;                                                        // coefficient of S g
          const float kg = -7.5f * q * ri7 + 1.5f * T * ri5;                                 // of g
          const float kd = -15.f * gsd * ri7 + 52.5f * q * gd * ri9 - 7.5f * T * gd * ri7;  // of d
          const float ks = -15.f * gd * ri7;                                                 // of S d
          vx += G * (kS * sgx + kg * gx[k] + kd * dx + ks * sdx);
          vy += G * (kS * sgy + kg * gy[k] + kd * dy + ks * sdy);
          vz += G * (kS * sgz + kg * gz[k] + kd * dz + ks * sdz);
          // sym(dL/dS)_ab = G [3/2 (g_a d_b + g_b d_a) / r^5 - 15/2 (g.d) d_a d_b / r^7 + 3/2 (g.d) delta_ab / r^5]
          const float a5 = 1.5f * ri5, b7 = -7.5f * gd * ri7, c5 = 1.5f * gd * ri5;
          hxx += 2.f * a5 * gx[k] * dx + b7 * dx * dx + c5;
          hyy += 2.f * a5 * gy[k] * dy + b7 * dy * dy + c5;
          hzz += 2.f * a5 * gz[k] * dz + b7 * dz * dz + c5;
          hxy += a5 * (gx[k] * dy + gy[k] * dx) + b7 * dx * dy;
          hxz += a5 * (gx[k] * dz + gz[k] * dx) + b7 * dx * dz;
          hyz += a5 * (gy[k] * dz + gz[k] * dy) + b7 * dy * dz;
        }
        tgx[k] += vx; tgy[k] += vy; tgz[k] += vz;
        gcx -= vx; gcy -= vy; gcz -= vz;
        gM = __builtin_fmaf(gd, ri3, gM);
      }
      if (valid) {
        // this lane owns visit n_first + e for every block of targets: the first block stores, the
        // later ones add (the same lane, in program order, so no atomics are needed)
        float4* q = A.vnode + (int64_t)(ORDER == 2 ? 3 : 1) * (tk.n_first + e);
        float4 v0 = make_float4(gcx, gcy, gcz, -G * gM);
        float4 v1 = make_float4(G * hxx, G * hyy, G * hzz, G * hxy), v2 = make_float4(G * hxz, G * hyz, 0.f, 0.f);
        if (tb0 > 0) {
          v0 += gld(q);
          if (ORDER == 2) {
            v1 += gld(q + 1);
            v2 += gld(q + 2);
          }
        }
        gst(q, v0);
        if (ORDER == 2) {
          gst(q + 1, v1);
          gst(q + 2, v2);
        }
      }
    }
    // ---- direct sources: lane = flat position within a group of up to 64 ranges
    int vbase = uniform(A.joff[t]);  // direct visit of the group's first flat position
    for (int rg = 0; rg < tk.j_nranges; rg += 64) {
      const int nr = tk.j_nranges - rg < 64 ? tk.j_nranges - rg : 64;
      int2 g = make_int2(0, 0);
      if (lane < nr) g = a.ranges[tk.j_first + rg + lane];
      int total;
      const int o = wave_excl_scan(g.y, &total);
      total = uniform(total);
      ro[wid][lane] = lane < nr ? o : 0x7fffffff;
      rb[wid][lane] = g.x;
      wave_sync();
      for (int f0 = wid * 64; f0 < total; f0 += W * 64) {
        const int f = f0 + lane;
        const bool valid = f < total;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        int sid = -2;
        if (valid) {
          // last range whose start offset is <= f (empty ranges share the next one's offset)
          int lo = 0, hi = nr - 1;
          while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (ro[wid][mid] <= f) lo = mid;
            else hi = mid - 1;
          }
          const int p = rb[wid][lo] + (f - ro[wid][lo]);
          s = a.rec[p];
          sid = PACKED ? A.src_id[p] : p;
        }
        const float Gm = G * s.w, m3 = -3.f * Gm;
        float gsx = 0.f, gsy = 0.f, gsz = 0.f, gms = 0.f;
#pragma unroll
        for (int k = 0; k < kTB; ++k) {
          if (k >= tb) break;  // (uniform) targets past the block's last do no work
          float ux = s.x - xt[k], uy = s.y - yt[k], uz = s.z - zt[k];
          float s2 = __builtin_fmaf(uz, uz, __builtin_fmaf(uy, uy, __builtin_fmaf(ux, ux, eps2)));
          float ri = __builtin_amdgcn_rsqf(s2);
          float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
          float gu = __builtin_fmaf(gz[k], uz, __builtin_fmaf(gy[k], uy, gx[k] * ux));
          const bool self = (sid == idt[k]);
          float c1 = self ? 0.f : Gm * ri3;
          float c2 = self ? 0.f : m3 * gu * ri5;
          float wx = __builtin_fmaf(c1, gx[k], c2 * ux);
          float wy = __builtin_fmaf(c1, gy[k], c2 * uy);
          float wz = __builtin_fmaf(c1, gz[k], c2 * uz);
          gsx += wx; gsy += wy; gsz += wz;
          tgx[k] -= wx; tgy[k] -= wy; tgz[k] -= wz;
          gms = __builtin_fmaf(self ? 0.f : gu, ri3, gms);
        }
        if (valid) {  // the lane's own direct visit, as for the nodes
          float4* q = A.vdir + (vbase + f);
          float4 v = make_float4(gsx, gsy, gsz, G * gms);
          if (tb0 > 0) v += gld(q);
          gst(q, v);
        }
      }
      vbase += total;
      wave_sync();
    }
    // ---- target gradients: reduce across the wavefront, one atomic per target component
#pragma unroll
    for (int k = 0; k < kTB; ++k) {
      float sx = wave_sum(tgx[k]), sy = wave_sum(tgy[k]), sz = wave_sum(tgz[k]);
      if (lane == k && k < tb) {
        float4* q = A.gpos + (tk.i_begin + tb0 + k);
        unsafeAtomicAdd(&q->x, sx);
        unsafeAtomicAdd(&q->y, sy);
        unsafeAtomicAdd(&q->z, sz);
      }
    }
    wave_sync();
  }
}

// One wavefront per chunk of a node's visits (at most kVisitChunk, in the node-sorted visit order):
// the chunk's sum, lanes striding the chunk, reduced across the wavefront in a fixed order.
template <int NQ>
__global__ void __launch_bounds__(256) k_visit_sum(const float4* __restrict__ vnode, const int32_t* __restrict__ nvis,
                                                   const int2* __restrict__ chunks, int32_t n_chunks,
                                                   float4* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int ch = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (ch >= n_chunks) return;
  const int2 r = gld(chunks + ch);
  float4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int i = r.x + lane; i < r.y; i += 64) {
    const float4* v = vnode + (int64_t)NQ * gld(nvis + i);
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += gld(v + q);
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float4 t = make_float4(wave_sum(acc[q].x), wave_sum(acc[q].y), wave_sum(acc[q].z), wave_sum(acc[q].w));
    if (lane == 0) gst(part + (int64_t)NQ * ch + q, t);
  }
}

// One workgroup per node (its member loop spread over 256 lanes: a top node holds tens of thousands of
// particles): its gradient (the sum of its chunks' sums, formed by each wavefront) pushed to the members:
// dx_k += (m_k / M) dL/dcom + 2 m_k H e_k, dm_k += dL/dM + e_k . dL/dcom / M + e_k.H e_k, e_k = x_k - com.
// A node whose member range is not inside [0, n_ids) is skipped and counted in *bad (its gradient is
// not pushed), so a malformed node table cannot make the member loop read or write out of bounds.
template <int NQ>
__global__ void __launch_bounds__(256) k_node_chain(const int32_t* __restrict__ node_range, int32_t n_nodes, const float4* __restrict__ nodes,
                             const float4* __restrict__ part, const int32_t* __restrict__ chunk_first,
                             const float4* __restrict__ rec_by_id, int32_t n_ids, float4* __restrict__ gpos,
                             float* __restrict__ gmass, int32_t* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  for (int nd = blockIdx.x; nd < n_nodes; nd += gridDim.x) {
    const int c0 = gld(chunk_first + nd), c1 = gld(chunk_first + nd + 1);
    if (c0 == c1) continue;  // the node is in no task's list
    const int b = node_range[2 * nd], n = node_range[2 * nd + 1];
    if (b < 0 || n < 0 || b > n_ids - n) {
      if (threadIdx.x == 0) atomicAdd(bad, 1);
      continue;
    }
    float4 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int ch = c0 + lane; ch < c1; ch += 64) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] += gld(part + (int64_t)NQ * ch + q);
    }
    float gv[4 * NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      gv[4 * q] = wave_sum(acc[q].x);
      gv[4 * q + 1] = wave_sum(acc[q].y);
      gv[4 * q + 2] = wave_sum(acc[q].z);
      gv[4 * q + 3] = wave_sum(acc[q].w);
    }
    const float4 c = nodes[3 * nd];
    const float invM = 1.f / c.w;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const float4 r = rec_by_id[b + k];
      const float f = r.w * invM;
      const float ex = r.x - c.x, ey = r.y - c.y, ez = r.z - c.z;
      float px = f * gv[0], py = f * gv[1], pz = f * gv[2];
      float dm = gv[3] + (ex * gv[0] + ey * gv[1] + ez * gv[2]) * invM;
      if constexpr (NQ == 3) {
        const float hxx = gv[4], hyy = gv[5], hzz = gv[6], hxy = gv[7], hxz = gv[8], hyz = gv[9];
        const float hx = hxx * ex + hxy * ey + hxz * ez;
        const float hy = hxy * ex + hyy * ey + hyz * ez;
        const float hz = hxz * ex + hyz * ey + hzz * ez;
        px += 2.f * r.w * hx;
        py += 2.f * r.w * hy;
        pz += 2.f * r.w * hz;
        dm += ex * hx + ey * hy + ez * hz;
      }
      float4* q = gpos + (b + k);
      unsafeAtomicAdd(&q->x, px);
      unsafeAtomicAdd(&q->y, py);
      unsafeAtomicAdd(&q->z, pz);
      unsafeAtomicAdd(gmass + (b + k), dm);
    }
  }
}

// One wavefront per 64 consecutive entries of the direct visits sorted by source id: a segmented
// inclusive scan (ids are sorted, so equal neighbours mean one run) sums each id's run within the
// wavefront, and the run's last lane adds it to the gradients.  A particle whose visits span several
// wavefronts gets one addition from each, so no lane walks a long list.
__global__ void __launch_bounds__(256) k_direct_sum(const float4* __restrict__ vdir, const int32_t* __restrict__ dvis,
                                                    const int32_t* __restrict__ dkey, int32_t n_vis,
                                                    float4* __restrict__ gpos, float* __restrict__ gmass) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n_vis;
  int key = valid ? gld(dkey + i) : -1 - lane;  // distinct negative keys: past-the-end lanes form no run
  float4 v = valid ? gld(vdir + gld(dvis + i)) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int ku = __shfl_up(key, d, 64);
    const float ux = __shfl_up(v.x, d, 64), uy = __shfl_up(v.y, d, 64), uz = __shfl_up(v.z, d, 64),
                uw = __shfl_up(v.w, d, 64);
    if (lane >= d && ku == key) {
      v.x += ux;
      v.y += uy;
      v.z += uz;
      v.w += uw;
    }
  }
  const int kn = __shfl_down(key, 1, 64);
  if (valid && (lane == 63 || kn != key)) {
    float4* q = gpos + key;
    unsafeAtomicAdd(&q->x, v.x);
    unsafeAtomicAdd(&q->y, v.y);
    unsafeAtomicAdd(&q->z, v.z);
    unsafeAtomicAdd(gmass + key, v.w);
  }
}

constexpr int kMaxTypes = 8;
constexpr int kLJTile = 128;

// Per-lane accumulators of dL/deps_ij and dL/dsigma_ij keyed by the j type (the lane's i type is
// fixed within a run chunk).  NT = 1 or 2 keep them in registers; NT = 0 (up to kMaxTypes types)
// adds each pair term to LDS directly.
template <int NT>
struct ParamAcc {
  float e[NT > 0 ? NT : 1], s[NT > 0 ? NT : 1];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < (NT > 0 ? NT : 1); ++k) e[k] = s[k] = 0.f;
  }
  __device__ __forceinline__ void add(int tj, float de, float ds, float* pg_row) {
    if (NT == 1) {
      e[0] += de;
      s[0] += ds;
    } else if (NT == 2) {
      const bool one = tj != 0;
      e[0] += one ? 0.f : de;
      s[0] += one ? 0.f : ds;
      e[1] += one ? de : 0.f;
      s[1] += one ? ds : 0.f;
    } else {
      atomicAdd(pg_row + 2 * tj, de);
      atomicAdd(pg_row + 2 * tj + 1, ds);
    }
  }
  __device__ __forceinline__ void flush(float* pg_row) {
    if (NT > 0) {
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (e[k] != 0.f) atomicAdd(pg_row + 2 * k, e[k]);
        if (s[k] != 0.f) atomicAdd(pg_row + 2 * k + 1, s[k]);
      }
    }
    zero();
  }
};

// The block's dL/deps_ij, dL/dsigma_ij by type pair (summed over its 4 wavefronts) go to its own
// row of A.ppart with plain stores; k_lj_param_reduce sums the rows in a fixed order.  (Atomics from
// every block onto the few words of gparam, all in one cache line, serialise at one L2 channel.)
__device__ __forceinline__ void block_param_partial(const LJAdjArgs& A, const float* pg, int nt) {
  const int P = 2 * nt * nt;
  if ((int)threadIdx.x < P) {
    float v = 0.f;
    for (int w = 0; w < 4; ++w) v += pg[w * 2 * kMaxTypes * kMaxTypes + threadIdx.x];
    A.ppart[(int64_t)blockIdx.x * P + threadIdx.x] = v;
  }
}

// One block per type pair (ta, tb): the sum of the blocks' partials, chained to the per-type
// parameters through eps_ij = sqrt(eps_a eps_b), sigma_ij = (sigma_a + sigma_b) / 2.
__global__ void __launch_bounds__(256) k_lj_param_reduce(const float* __restrict__ ppart, int32_t n_blocks, int32_t nt,
                                                         const float* __restrict__ eps_t, float* __restrict__ gparam) {
  __shared__ float se[256], ss[256];
  const int k = blockIdx.x, P = 2 * nt * nt;
  float de = 0.f, ds = 0.f;
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) {
    de += ppart[(int64_t)b * P + 2 * k];
    ds += ppart[(int64_t)b * P + 2 * k + 1];
  }
  se[threadIdx.x] = de;
  ss[threadIdx.x] = ds;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      se[threadIdx.x] += se[threadIdx.x + h];
      ss[threadIdx.x] += ss[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int ta = k / nt, tb = k % nt;
    const float eij = sqrtf(eps_t[ta] * eps_t[tb]);
    unsafeAtomicAdd(gparam + ta, se[0] * eps_t[tb] / (2.f * eij));
    unsafeAtomicAdd(gparam + tb, se[0] * eps_t[ta] / (2.f * eij));
    unsafeAtomicAdd(gparam + nt + ta, 0.5f * ss[0]);
    unsafeAtomicAdd(gparam + nt + tb, 0.5f * ss[0]);
  }
}

// One wavefront per run of tasks sharing a target range (as in the forward kernel); lanes =
// (i atom) x (j slice) with a per-lane rotation over the slice's j entries.  j-side gradients and
// forces accumulate in LDS, i-side in registers across the run.
template <int NT>
__global__ void __launch_bounds__(256) k_lj_adj(LJAdjArgs A) {
  const LJArgs& a = A.f;
  __shared__ float2 tab[kMaxTypes * kMaxTypes];   // (24 eps_ij, sigma_ij)
  __shared__ float4 jt[4][kLJTile], jh[4][kLJTile];
  __shared__ float gj[4][6][kLJTile];              // j: dL/dx (3), force (3)
  __shared__ float red[4][6][64];
  __shared__ float pg[4][2 * kMaxTypes * kMaxTypes];  // per wave: dL/deps_ij, dL/dsigma_ij by type pair
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int nt = a.n_types;
  for (int k = threadIdx.x; k < nt * nt; k += blockDim.x) {
    int ta = k / nt, tb = k % nt;
    tab[k] = make_float2(24.f * sqrtf(a.eps_t[ta] * a.eps_t[tb]), 0.5f * (a.sig_t[ta] + a.sig_t[tb]));
  }
  for (int k = threadIdx.x; k < 4 * 2 * kMaxTypes * kMaxTypes; k += blockDim.x) (&pg[0][0])[k] = 0.f;
  __syncthreads();
  const int r = uniform(blockIdx.x * 4 + wid);
  if (r < a.n_runs) {
    const int t0 = uniform(a.runs[r]), t1 = uniform(a.runs[r + 1]);
    const gc_task tk0 = a.tasks[t0];
    const int ipos0 = a.ibeg ? a.ibeg[t0] : tk0.i_begin;
    for (int i0 = 0; i0 < tk0.i_count; i0 += 64) {
      const int icc = tk0.i_count - i0 < 64 ? tk0.i_count - i0 : 64;
      const int S = 64 / icc;
      const int il = lane % icc, sl = lane / icc;
      const bool active = sl < S;
      float xr = 0.f, yr = 0.f, zr = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
      int ti = 0;
      if (active) {
        float4 rr = a.rec[ipos0 + i0 + il];
        xr = rr.x; yr = rr.y; zr = rr.z;
        ti = (int)rr.w;
        float4 g = A.cot[tk0.i_begin + i0 + il];
        float m = A.mass_t[ti];
        hx = g.x / m; hy = g.y / m; hz = g.z / m;
      }
      float* pg_row = &pg[wid][2 * ti * nt];
      ParamAcc<NT> pa;
      pa.zero();
      float Gx = 0.f, Gy = 0.f, Gz = 0.f, Fx = 0.f, Fy = 0.f, Fz = 0.f;
      for (int t = t0; t < t1; ++t) {
        const gc_task tk = a.tasks[t];
        const int2 gjr = a.ranges[tk.j_first];
        const int2 gjid = a.ranges_id[tk.j_first];
        const bool self = (tk.flags & GC_TASK_SELF) != 0;
        const float xi = xr - (tk.shift[0] > 0.f ? tk.shift[0] : 0.f);
        const float yi = yr - (tk.shift[1] > 0.f ? tk.shift[1] : 0.f);
        const float zi = zr - (tk.shift[2] > 0.f ? tk.shift[2] : 0.f);
        const float sb0 = tk.shift[0] < 0.f ? tk.shift[0] : 0.f;
        const float sb1 = tk.shift[1] < 0.f ? tk.shift[1] : 0.f;
        const float sb2 = tk.shift[2] < 0.f ? tk.shift[2] : 0.f;
        for (int j0 = 0; j0 < gjr.y; j0 += kLJTile) {
          const int cnt = gjr.y - j0 < kLJTile ? gjr.y - j0 : kLJTile;
          for (int e = lane; e < cnt; e += 64) {
            float4 rj = a.rec[gjr.x + j0 + e];
            jt[wid][e] = make_float4(rj.x + sb0, rj.y + sb1, rj.z + sb2, rj.w);
            float4 g = A.cot[gjid.x + j0 + e];
            float m = A.mass_t[(int)rj.w];
            jh[wid][e] = make_float4(g.x / m, g.y / m, g.z / m, 0.f);
#pragma unroll
            for (int q = 0; q < 6; ++q) gj[wid][q][e] = 0.f;
          }
          wave_sync();
          if (active) {
            const int C = (cnt + S - 1) / S;
            const int e0 = sl * C, e1 = e0 + C < cnt ? e0 + C : cnt;
            const int cs = e1 - e0;
            if (cs > 0) {
              int e = e0 + il % cs;
              for (int k = 0; k < cs; ++k) {
                if (!(self && j0 + e <= i0 + il)) {
                  const float4 j = jt[wid][e];
                  const float dx = xi - j.x, dy = yi - j.y, dz = zi - j.z;
                  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                  if (r2 < a.rc2) {
                    const int tj = (int)j.w;
                    const float2 p = tab[ti * nt + tj];
                    const float e24 = p.x, sg = p.y;
                    const float ri2 = __builtin_amdgcn_rcpf(r2);
                    const float q = sg * sg * ri2;
                    const float q3 = q * q * q;
                    const float f = e24 * q3 * __builtin_fmaf(2.f, q3, -1.f) * ri2;          // force factor
                    const float fp = e24 * q3 * __builtin_fmaf(-14.f, q3, 4.f) * ri2 * ri2;  // df / d(r^2)
                    const float4 hj = jh[wid][e];
                    const float dhx = hx - hj.x, dhy = hy - hj.y, dhz = hz - hj.z;
                    const float pp = __builtin_fmaf(dhz, dz, __builtin_fmaf(dhy, dy, dhx * dx));
                    const float c2 = 2.f * fp * pp;
                    const float wx = __builtin_fmaf(f, dhx, c2 * dx);
                    const float wy = __builtin_fmaf(f, dhy, c2 * dy);
                    const float wz = __builtin_fmaf(f, dhz, c2 * dz);
                    Gx += wx; Gy += wy; Gz += wz;
                    Fx = __builtin_fmaf(f, dx, Fx);
                    Fy = __builtin_fmaf(f, dy, Fy);
                    Fz = __builtin_fmaf(f, dz, Fz);
                    atomicAdd(&gj[wid][0][e], -wx);
                    atomicAdd(&gj[wid][1][e], -wy);
                    atomicAdd(&gj[wid][2][e], -wz);
                    atomicAdd(&gj[wid][3][e], -f * dx);
                    atomicAdd(&gj[wid][4][e], -f * dy);
                    atomicAdd(&gj[wid][5][e], -f * dz);
                    // dL/deps_ij = p f / eps_ij; dL/dsigma_ij = p (24 eps)(24 s^11 r^-14 - 6 s^5 r^-8)
                    const float dle = pp * f * 24.f / e24;
                    const float fs = e24 * q3 * __builtin_fmaf(24.f, q3, -6.f) * ri2 / sg;
                    pa.add(tj, dle, pp * fs, pg_row);
                  }
                }
                e = (e + 1 == e1) ? e0 : e + 1;
              }
            }
          }
          wave_sync();
          for (int e = lane; e < cnt; e += 64) {
            const int id = gjid.x + j0 + e;
            float4* q = A.gpos + id;
            unsafeAtomicAdd(&q->x, gj[wid][0][e]);
            unsafeAtomicAdd(&q->y, gj[wid][1][e]);
            unsafeAtomicAdd(&q->z, gj[wid][2][e]);
            float4* fq = A.force + id;
            unsafeAtomicAdd(&fq->x, gj[wid][3][e]);
            unsafeAtomicAdd(&fq->y, gj[wid][4][e]);
            unsafeAtomicAdd(&fq->z, gj[wid][5][e]);
          }
          wave_sync();
        }
      }
      if (active) pa.flush(pg_row);
      red[wid][0][lane] = Gx; red[wid][1][lane] = Gy; red[wid][2][lane] = Gz;
      red[wid][3][lane] = Fx; red[wid][4][lane] = Fy; red[wid][5][lane] = Fz;
      wave_sync();
      if (lane < icc) {
        float sm[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int sidx = 0; sidx < S; ++sidx)
#pragma unroll
          for (int q = 0; q < 6; ++q) sm[q] += red[wid][q][sidx * icc + lane];
        const int id = tk0.i_begin + i0 + lane;
        float4* q = A.gpos + id;
        unsafeAtomicAdd(&q->x, sm[0]);
        unsafeAtomicAdd(&q->y, sm[1]);
        unsafeAtomicAdd(&q->z, sm[2]);
        float4* fq = A.force + id;
        unsafeAtomicAdd(&fq->x, sm[3]);
        unsafeAtomicAdd(&fq->y, sm[4]);
        unsafeAtomicAdd(&fq->z, sm[5]);
      }
      wave_sync();
    }
  }
  __syncthreads();
  block_param_partial(A, &pg[0][0], nt);
}

// Gather form of the Lennard-Jones adjoint (see the forward gather form for the schedule and the
// cutoff arithmetic).  Each target atom's dL/dx is added to gpos and its recomputed force written
// to `force` by one wavefront; the parameter derivatives go through per-lane sums keyed by the
// source type, the block's LDS, then one atomic per type pair and block.
constexpr int kGTile = 64;   // source records per LDS tile per wavefront
constexpr int kEGroup = 32;  // tasks whose sources a wavefront stages at a time
constexpr float kFar = 1e18f;

template <int NT, bool SHIFTED>
__device__ __forceinline__ void adj_gather_tile(const float4* __restrict__ p, const float4* __restrict__ hp,
                                                const float4* __restrict__ o, int C, float tx, float ty, float tz,
                                                float hx, float hy, float hz, const float4* __restrict__ trow,
                                                float4 p0, float rc2, float (&acc)[6], ParamAcc<NT>& pa,
                                                float* pg_row) {
  for (int k = 0; k < C; ++k) {
    const float4 sj = p[k], hj = hp[k];
    float ux = tx, uy = ty, uz = tz;
    if (SHIFTED) {
      const float4 w = o[k];
      ux = tx + w.x;
      uy = ty + w.y;
      uz = tz + w.z;
    }
    const float ex = ux - sj.x, ey = uy - sj.y, ez = uz - sj.z;
    const float r2 = __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex));
    const bool in = r2 < rc2 && r2 > 0.f;
    const int tj = (int)sj.w;
    const float4 c = NT == 1 ? p0 : trow[tj];  // (24 eps_ij, sigma_ij, 12 / (24 eps_ij), 1 / sigma_ij)
    const float ri2 = __builtin_amdgcn_rcpf(r2);
    const float q = c.y * c.y * ri2;
    const float q3 = q * q * q;
    const float eq = c.x * q3;
    float f = eq * __builtin_fmaf(2.f, q3, -1.f) * ri2;                  // force factor
    float fp = eq * __builtin_fmaf(-14.f, q3, 4.f) * ri2 * ri2;          // df / d(r^2)
    float fs = eq * __builtin_fmaf(12.f, q3, -3.f) * ri2 * c.w;          // half of d(f r^2 ...)/dsigma term
    f = in ? f : 0.f;
    fp = in ? fp : 0.f;
    fs = in ? fs : 0.f;
    const float dhx = hx - hj.x, dhy = hy - hj.y, dhz = hz - hj.z;
    const float pp = __builtin_fmaf(dhz, ez, __builtin_fmaf(dhy, ey, dhx * ex));
    const float c2 = 2.f * fp * pp;
    acc[0] += __builtin_fmaf(f, dhx, c2 * ex);
    acc[1] += __builtin_fmaf(f, dhy, c2 * ey);
    acc[2] += __builtin_fmaf(f, dhz, c2 * ez);
    acc[3] = __builtin_fmaf(f, ex, acc[3]);
    acc[4] = __builtin_fmaf(f, ey, acc[4]);
    acc[5] = __builtin_fmaf(f, ez, acc[5]);
    pa.add(tj, pp * f * c.z, pp * fs, pg_row);
  }
}

template <int NT>
__global__ void __launch_bounds__(256) k_lj_adj_gather(LJAdjArgs A) {
  const LJArgs& a = A.f;
  __shared__ float4 tab[kMaxTypes * kMaxTypes];
  // per wavefront: sources, their g / m, their target-side shifts; the slice reduction at the end
  // reuses the area
  __shared__ float4 sbuf[4][3 * kGTile];
  __shared__ float4 esh[4][kEGroup], eto[4][kEGroup];
  __shared__ int eoff[4][kEGroup], ebeg[4][kEGroup], ebid[4][kEGroup];
  __shared__ float pg[4][2 * kMaxTypes * kMaxTypes];
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  float4* src = sbuf[wid];
  float4* hsr = sbuf[wid] + kGTile;
  float4* tof = sbuf[wid] + 2 * kGTile;
  float* red = reinterpret_cast<float*>(sbuf[wid]);  // 6 x 64 floats
  static_assert(3 * kGTile * 4 >= 6 * 64, "reduction area");
  const int nt = a.n_types;
  for (int k = threadIdx.x; k < nt * nt; k += blockDim.x) {
    const int ta = k / nt, tb = k % nt;
    const float e24 = 24.f * sqrtf(a.eps_t[ta] * a.eps_t[tb]), sg = 0.5f * (a.sig_t[ta] + a.sig_t[tb]);
    tab[k] = make_float4(e24, sg, 12.f / e24, 1.f / sg);
  }
  for (int k = threadIdx.x; k < 4 * 2 * kMaxTypes * kMaxTypes; k += blockDim.x) (&pg[0][0])[k] = 0.f;
  __syncthreads();
  const float4 p0 = tab[0];
  const int32_t* tw0 = reinterpret_cast<const int32_t*>(a.tasks);
  constexpr int kTaskWords = sizeof(gc_task) / 4;
  const int g = uniform(blockIdx.x * 4 + wid);
  if (g < a.n_tgt) {
    const int4 tg = dev::gld(a.tgt + g);
    const int id0 = uniform(tg.x), cnt = uniform(tg.y), e0 = uniform(tg.z), ne = uniform(tg.w);
    const int en0 = uniform(dev::gld(a.ent + e0));
    const int32_t* tw = tw0 + (int64_t)(en0 >> 1) * kTaskWords;
    const int rb = (en0 & 1) ? uniform(dev::gld(a.ranges + uniform(dev::gld(tw + 2))).x)
                             : (a.ibeg ? uniform(dev::gld(a.ibeg + (en0 >> 1))) : uniform(dev::gld(tw)));
    for (int i0 = 0; i0 < cnt; i0 += 64) {
      const int icc = cnt - i0 < 64 ? cnt - i0 : 64;
      const int S = 64 / icc;
      const int il = lane % icc, sl = lane / icc;
      const bool active = sl < S;
      float tx = 0.f, ty = 0.f, tz = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
      int ti = 0;
      if (active) {
        const float4 r = dev::gld(a.rec + rb + i0 + il);
        tx = r.x; ty = r.y; tz = r.z;
        ti = (int)r.w;
        const float4 gc4 = dev::gld(A.cot + id0 + i0 + il);
        const float m = A.mass_t[ti];
        hx = gc4.x / m; hy = gc4.y / m; hz = gc4.z / m;
      }
      const float4* trow = tab + ti * nt;
      float* pg_row = &pg[wid][2 * ti * nt];
      ParamAcc<NT> pa;
      pa.zero();
      float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const int DT = S * (kGTile / S);
      // candidates pruned against the targets' bounding box as in the forward gather (every term of a
      // pair outside the cutoff is zero, so a source beyond r_c of the box adds nothing)
      const float blx = wave_min(active ? tx : kFar), bly = wave_min(active ? ty : kFar),
                  blz = wave_min(active ? tz : kFar);
      const float bhx = wave_max(active ? tx : -kFar), bhy = wave_max(active ? ty : -kFar),
                  bhz = wave_max(active ? tz : -kFar);
      const float keep2 = a.rc2 * 1.001f;
      for (int eg = 0; eg < ne; eg += kEGroup) {
        const int nen = ne - eg < kEGroup ? ne - eg : kEGroup;
        int n = 0, sb = 0, sid = 0;
        float4 sh = make_float4(0.f, 0.f, 0.f, 0.f), to = sh;
        if (lane < nen) {
          const int en = dev::gld(a.ent + e0 + eg + lane);
          const int t = en >> 1;
          const int32_t* w = tw0 + (int64_t)t * kTaskWords;
          const float s0 = __int_as_float(dev::gld(w + 7)), s1 = __int_as_float(dev::gld(w + 8)),
                      s2 = __int_as_float(dev::gld(w + 9));
          const float ax = s0 > 0.f ? s0 : 0.f, ay = s1 > 0.f ? s1 : 0.f, az = s2 > 0.f ? s2 : 0.f;
          const float bx = s0 < 0.f ? s0 : 0.f, by = s1 < 0.f ? s1 : 0.f, bz = s2 < 0.f ? s2 : 0.f;
          if (en & 1) {
            sb = a.ibeg ? dev::gld(a.ibeg + t) : dev::gld(w);
            sid = dev::gld(w);
            n = dev::gld(w + 1);
            sh = make_float4(-ax, -ay, -az, 0.f);
            to = make_float4(bx, by, bz, 0.f);
          } else {
            const int jf = dev::gld(w + 2);
            const int2 jr = dev::gld(a.ranges + jf);
            sb = jr.x;
            sid = dev::gld(a.ranges_id + jf).x;
            n = jr.y;
            sh = make_float4(bx, by, bz, 0.f);
            to = make_float4(-ax, -ay, -az, 0.f);
          }
        }
        int total;
        const int off = dev::wave_excl_scan(n, &total);
        total = uniform(total);
        const bool shifted = __ballot(lane < nen && (to.x != 0.f || to.y != 0.f || to.z != 0.f)) != 0ull;
        if (lane < kEGroup) {
          eoff[wid][lane] = lane < nen ? off : 0x7fffffff;
          ebeg[wid][lane] = sb;
          ebid[wid][lane] = sid;
          esh[wid][lane] = sh;
          eto[wid][lane] = to;
        }
        wave_sync();
        for (int ws = 0; ws < total; ws += DT) {
          // one source per lane (DT <= 64): staged, tested, and the survivors compacted
          const int c = total - ws < DT ? total - ws : DT;
          float4 v = make_float4(kFar, kFar, kFar, 0.f), hv = make_float4(0.f, 0.f, 0.f, 0.f), o = hv;
          bool keep = false;
          if (lane < c) {
            const int f = ws + lane;
            int lo = 0, hi = nen - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (eoff[wid][mid] <= f) lo = mid;
              else hi = mid - 1;
            }
            const int k = f - eoff[wid][lo];
            const float4 r = dev::gld(a.rec + ebeg[wid][lo] + k);
            const float4 q = esh[wid][lo];
            v = make_float4(r.x + q.x, r.y + q.y, r.z + q.z, r.w);
            o = eto[wid][lo];
            const float px = v.x - o.x, py = v.y - o.y, pz = v.z - o.z;
            const float dx = fmaxf(fmaxf(blx - px, px - bhx), 0.f);
            const float dy = fmaxf(fmaxf(bly - py, py - bhy), 0.f);
            const float dz = fmaxf(fmaxf(blz - pz, pz - bhz), 0.f);
            keep = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)) <= keep2;
            if (keep) {
              const float4 gs = dev::gld(A.cot + ebid[wid][lo] + k);
              const float ms = A.mass_t[(int)r.w];
              hv = make_float4(gs.x / ms, gs.y / ms, gs.z / ms, 0.f);
            }
          }
          const uint64_t km = __ballot(keep);
          const int kc = uniform(__popcll(km));
          const int C = (kc + S - 1) / S;
          const int padded = S * C;
          if (keep) {
            const int kk = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
            src[kk] = v;
            hsr[kk] = hv;
            if (shifted) tof[kk] = o;
          }
          if (lane >= kc && lane < padded) {
            src[lane] = make_float4(kFar, kFar, kFar, 0.f);
            hsr[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (shifted) tof[lane] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
          wave_sync();
          if (active && C > 0) {
            if (shifted)
              adj_gather_tile<NT, true>(src + sl * C, hsr + sl * C, tof + sl * C, C, tx, ty, tz, hx,
                                        hy, hz, trow, p0, a.rc2, acc, pa, pg_row);
            else
              adj_gather_tile<NT, false>(src + sl * C, hsr + sl * C, nullptr, C, tx, ty, tz, hx, hy, hz,
                                         trow, p0, a.rc2, acc, pa, pg_row);
          }
          wave_sync();
        }
      }
      if (active) pa.flush(pg_row);
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q * 64 + lane] = acc[q];
      wave_sync();
      if (lane < icc) {
        float sm[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int sidx = 0; sidx < S; ++sidx)
#pragma unroll
          for (int q = 0; q < 6; ++q) sm[q] += red[q * 64 + sidx * icc + lane];
        const int id = id0 + i0 + lane;
        const float4 g0 = dev::gld(A.gpos + id);
        dev::gst(A.gpos + id, make_float4(g0.x + sm[0], g0.y + sm[1], g0.z + sm[2], g0.w));
        dev::gst(A.force + id, make_float4(sm[3], sm[4], sm[5], 0.f));
      }
      wave_sync();
    }
  }
  __syncthreads();
  block_param_partial(A, &pg[0][0], nt);
}

__global__ void k_lj_mass_grad(const float4* __restrict__ cot, const float4* __restrict__ force,
                               const float* __restrict__ mass_t, const float4* __restrict__ rec_by_id,
                               float* __restrict__ gmass, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float4 g = cot[i], F = force[i];
    const float m = mass_t[(int)rec_by_id[i].w];
    gmass[i] += -(g.x * F.x + g.y * F.y + g.z * F.z) / (m * m);
  }
}

}  // namespace

hipError_t launch_grav_adjoint(bool packed, int order, const GravAdjArgs& a, int wpb, hipStream_t s) {
  if (a.f.n_tasks <= 0) return hipSuccess;
  if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
  const int grid = a.f.n_tasks;
  const dim3 block(64 * wpb);
  if (order == 2) {
    if (packed) hipLaunchKernelGGL((k_grav_adj<true, 2>), dim3(grid), block, 0, s, a);
    else hipLaunchKernelGGL((k_grav_adj<false, 2>), dim3(grid), block, 0, s, a);
  } else {
    if (packed) hipLaunchKernelGGL((k_grav_adj<true, 1>), dim3(grid), block, 0, s, a);
    else hipLaunchKernelGGL((k_grav_adj<false, 1>), dim3(grid), block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_visit_sums(int order, const float4* vnode, const int32_t* nvis, const int2* chunks,
                             int32_t n_chunks, float4* part, hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  const int g = (n_chunks + 3) / 4;
  if (order == 2)
    hipLaunchKernelGGL(k_visit_sum<3>, dim3(g), dim3(256), 0, s, vnode, nvis, chunks, n_chunks, part);
  else
    hipLaunchKernelGGL(k_visit_sum<1>, dim3(g), dim3(256), 0, s, vnode, nvis, chunks, n_chunks, part);
  return hipGetLastError();
}

hipError_t launch_node_chain(int order, const int32_t* node_range, int32_t n_nodes, const float4* nodes,
                             const float4* part, const int32_t* chunk_first, const float4* rec_by_id, int32_t n_ids,
                             float4* gpos, float* gmass, int32_t* bad, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  const int g = n_nodes < 65536 ? n_nodes : 65536;
  if (order == 2)
    hipLaunchKernelGGL(k_node_chain<3>, dim3(g), dim3(256), 0, s, node_range, n_nodes, nodes, part, chunk_first,
                       rec_by_id, n_ids, gpos, gmass, bad);
  else
    hipLaunchKernelGGL(k_node_chain<1>, dim3(g), dim3(256), 0, s, node_range, n_nodes, nodes, part, chunk_first,
                       rec_by_id, n_ids, gpos, gmass, bad);
  return hipGetLastError();
}

hipError_t launch_direct_sums(const float4* vdir, const int32_t* dvis, const int32_t* dkey, int32_t n_vis,
                              float4* gpos, float* gmass, hipStream_t s) {
  if (n_vis <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_direct_sum, dim3((n_vis + 255) / 256), dim3(256), 0, s, vdir, dvis, dkey, n_vis, gpos, gmass);
  return hipGetLastError();
}

int lj_adjoint_blocks(const LJArgs& f, bool gather) { return gather ? (f.n_tgt + 3) / 4 : (f.n_runs + 3) / 4; }

hipError_t launch_lj_adjoint(const LJAdjArgs& a, int wpb, hipStream_t s) {
  (void)wpb;
  if (a.f.n_runs <= 0) return hipSuccess;
  const int nb = lj_adjoint_blocks(a.f, false);
  if (a.f.n_types == 1) hipLaunchKernelGGL(k_lj_adj<1>, dim3(nb), dim3(256), 0, s, a);
  else if (a.f.n_types == 2) hipLaunchKernelGGL(k_lj_adj<2>, dim3(nb), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_lj_adj<0>, dim3(nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_lj_param_reduce, dim3(a.f.n_types * a.f.n_types), dim3(256), 0, s, a.ppart, nb, a.f.n_types,
                     a.f.eps_t, a.gparam);
  return hipGetLastError();
}

hipError_t launch_lj_adjoint_gather(const LJAdjArgs& a, hipStream_t s) {
  if (a.f.n_tgt <= 0) return hipSuccess;
  const int nb = lj_adjoint_blocks(a.f, true);
  if (a.f.n_types == 1) hipLaunchKernelGGL(k_lj_adj_gather<1>, dim3(nb), dim3(256), 0, s, a);
  else if (a.f.n_types == 2) hipLaunchKernelGGL(k_lj_adj_gather<2>, dim3(nb), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_lj_adj_gather<0>, dim3(nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_lj_param_reduce, dim3(a.f.n_types * a.f.n_types), dim3(256), 0, s, a.ppart, nb, a.f.n_types,
                     a.f.eps_t, a.gparam);
  return hipGetLastError();
}

hipError_t launch_lj_mass_grad(const float4* cot, const float4* force, const float* mass_t, const float4* rec_by_id,
                               float* gmass, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_lj_mass_grad, dim3(g), dim3(256), 0, s, cot, force, mass_t, rec_by_id, gmass, n);
  return hipGetLastError();
}

}  // namespace gc
