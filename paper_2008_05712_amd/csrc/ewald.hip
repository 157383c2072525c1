// Combined Ewald kernel: the correction of periodic gravity (Sec. 4.1: ChaNGa sums the periodic
// images by Ewald summation on the GPU; Sec. 4.3: its work requests are combined like the force
// requests).  Every target of every task of a batch in one launch.
//
// For a cubic box of side L holding total mass M with centre of mass c, at r = x - c (nearest
// image) and splitting parameter alpha, the correction is the pull of every periodic image of M
// plus the neutralising background, less the central copy's direct pull (the tree walk computes
// that one):
//   a = G M [ sum_{n != 0, |n_d| <= nrep} -(erfc(alpha s)/s^3 + 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec
//           + (erf(alpha s)/s^3 - 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec          (n = 0)
//           - 2/L^2 sum_{0 < |h|^2 <= hmax2} e^{-pi^2 |h|^2/(alpha L)^2}/|h|^2 sin(2 pi h.r/L) h ],
// s_vec = r + n L.  The n = 0 bracket cancels near s = 0 and is taken there from its Taylor series
// in x = alpha s: 2/sqrt(pi) (2/3 - 2/5 x^2 + 1/7 x^4 - 1/27 x^6 + 1/132 x^8) alpha^3.
//
// With the box's second moment S about c the same kernel is expanded to second order: each image
// adds G [1/2 (tr(S) s_vec + 2 S s_vec) B_2 - 1/2 (s_vec.S.s_vec) s_vec B_3], with the radial
// derivatives B_l = ((2l - 1) B_{l-1} + (2 alpha^2)^l / (alpha sqrt(pi)) e^{-alpha^2 s^2}) / s^2 of
// B_0 = erfc(alpha s)/s (n != 0) or -erf(alpha s)/s (n = 0, from its series below alpha s = 1:
// -(2/sqrt(pi)) 2^l alpha^{2l+1} sum_j (-1)^j x^{2j} / (j! (2j + 2l + 1))), and each wave vector adds
// G 4 pi^2/L^4 e^{-pi^2 |h|^2/(alpha L)^2}/|h|^2 (h.S.h) sin(2 pi h.r/L) h, which is target independent
// apart from the sine and so joins the monopole's weight in the table.
//
// A bucket holds about ten targets and each target costs thousands of VALU operations, so the lanes
// take the batch's targets in flat order (a lane finds its task by binary search over the per-task
// target offsets) rather than one workgroup per bucket, which would leave most of a wave64 idle.
// The wave-vector terms h and -h are equal (sin is odd), so the table keeps one of each pair with
// twice the weight; each block builds it in LDS in a fixed order.  sin(2 pi t) is sinpi(2 t).
#include "gc_internal.h"
#include "mem_dev.h"

namespace gc {
namespace {

constexpr int kEwThreads = 256;

// sum_{j <= 10} (-1)^j x2^j / (j! (2j + 2l + 1)) for l = 2, 3 (Horner; the next term is below 1e-8
// of the first for x2 < 1)
__device__ __forceinline__ float erf_series_2(float x2) {
  float p = 1.f / 90720000.f;
  p = __builtin_fmaf(p, x2, -1.f / 8346240.f);
  p = __builtin_fmaf(p, x2, 1.f / 846720.f);
  p = __builtin_fmaf(p, x2, -1.f / 95760.f);
  p = __builtin_fmaf(p, x2, 1.f / 12240.f);
  p = __builtin_fmaf(p, x2, -1.f / 1800.f);
  p = __builtin_fmaf(p, x2, 1.f / 312.f);
  p = __builtin_fmaf(p, x2, -1.f / 66.f);
  p = __builtin_fmaf(p, x2, 1.f / 18.f);
  p = __builtin_fmaf(p, x2, -1.f / 7.f);
  return __builtin_fmaf(p, x2, 1.f / 5.f);
}
__device__ __forceinline__ float erf_series_3(float x2) {
  float p = 1.f / 97977600.f;
  p = __builtin_fmaf(p, x2, -1.f / 9072000.f);
  p = __builtin_fmaf(p, x2, 1.f / 927360.f);
  p = __builtin_fmaf(p, x2, -1.f / 105840.f);
  p = __builtin_fmaf(p, x2, 1.f / 13680.f);
  p = __builtin_fmaf(p, x2, -1.f / 2040.f);
  p = __builtin_fmaf(p, x2, 1.f / 360.f);
  p = __builtin_fmaf(p, x2, -1.f / 78.f);
  p = __builtin_fmaf(p, x2, 1.f / 22.f);
  p = __builtin_fmaf(p, x2, -1.f / 9.f);
  return __builtin_fmaf(p, x2, 1.f / 7.f);
}

template <bool QUAD>
__global__ void __launch_bounds__(kEwThreads) k_ewald(EwaldArgs a) {
  __shared__ float4 htab[kEwaldMaxH];  // (hx, hy, hz, weight)
  __shared__ int s_nh;
  const int lane = threadIdx.x & 63;
  // wave 0 lists the half-space wave vectors 0 < |h|^2 <= hmax2 in cube order, compacted by ballot
  if (threadIdx.x < 64) {
    const int hm = a.hmax;
    const int side = 2 * hm + 1, ncand = side * side * side;
    int cnt = 0;
    for (int b = 0; b < ncand; b += 64) {
      const int c = b + lane;
      int hx = 0, hy = 0, hz = 0;
      bool keep = false;
      if (c < ncand) {
        hx = c / (side * side) - hm;
        hy = (c / side) % side - hm;
        hz = c % side - hm;
        const int h2 = hx * hx + hy * hy + hz * hz;
        const bool upper = hx > 0 || (hx == 0 && (hy > 0 || (hy == 0 && hz > 0)));
        keep = upper && h2 <= a.hmax2;
      }
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int k = cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const float h2 = (float)(hx * hx + hy * hy + hz * hz);
        float kc = a.kcoef;
        if (QUAD) {
          const float fx = (float)hx, fy = (float)hy, fz = (float)hz;
          const float hSh = fx * (a.GS[0] * fx + a.GS[3] * fy + a.GS[4] * fz) +
                            fy * (a.GS[3] * fx + a.GS[1] * fy + a.GS[5] * fz) +
                            fz * (a.GS[4] * fx + a.GS[5] * fy + a.GS[2] * fz);
          kc = __builtin_fmaf(a.qcoef, hSh, kc);
        }
        const float w = 2.f * kc * expf(-a.kdecay * h2) / h2;  // both h and -h
        htab[k] = make_float4((float)hx, (float)hy, (float)hz, w);
      }
      cnt += __popcll(m);
    }
    if (lane == 0) s_nh = cnt;
  }
  __syncthreads();
  const int nh = s_nh;
  const int64_t f = (int64_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (f >= a.n_targets) return;
  // this lane's task: the last with ioff[t] <= f
  int lo = 0, hi = a.n_tasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (dev::gld(a.ioff + mid) <= f) lo = mid;
    else hi = mid - 1;
  }
  const int k = (int)(f - dev::gld(a.ioff + lo));
  const int32_t* tw = reinterpret_cast<const int32_t*>(a.tasks + lo);
  const int id = dev::gld(tw) + k;
  const int pos = (a.ibeg ? dev::gld(a.ibeg + lo) : dev::gld(tw)) + k;
  const float4 x = dev::gld(a.rec + pos);
  float r[3] = {x.x - a.c[0], x.y - a.c[1], x.z - a.c[2]};
#pragma unroll
  for (int d = 0; d < 3; ++d) r[d] -= a.L * rintf(r[d] * a.inv_L);
  const float al = a.alpha, sp = 1.1283791670955126f * al;  // 2 alpha / sqrt(pi)
  const float al2 = al * al, k2 = 2.f * al2 * sp, k3 = 4.f * al2 * al2 * sp;  // (2 alpha^2)^l / (alpha sqrt(pi))
  const float d2c = -4.f * sp * al2 * al2, d3c = 2.f * d2c * al2;  // -(2/sqrt(pi)) 2^l alpha^{2l+1}
  const float tr = a.GS[0] + a.GS[1] + a.GS[2];
  float ax = 0.f, ay = 0.f, az = 0.f, qx = 0.f, qy = 0.f, qz = 0.f;
  for (int nx = -a.nrep; nx <= a.nrep; ++nx)
    for (int ny = -a.nrep; ny <= a.nrep; ++ny)
      for (int nz = -a.nrep; nz <= a.nrep; ++nz) {
        const float sx = r[0] + (float)nx * a.L, sy = r[1] + (float)ny * a.L, sz = r[2] + (float)nz * a.L;
        const float s2 = __builtin_fmaf(sz, sz, __builtin_fmaf(sy, sy, sx * sx));
        const float s = sqrtf(s2);
        const float xs = al * s;
        float kf, b2 = 0.f, b3 = 0.f;  // kf = -B_1
        if (nx == 0 && ny == 0 && nz == 0) {
          const float x2 = xs * xs;
          if (xs < 0.5f) {
            kf = 1.1283791670955126f * al * al * al *
                 (2.f / 3.f + x2 * (-2.f / 5.f + x2 * (1.f / 7.f + x2 * (-1.f / 27.f + x2 * (1.f / 132.f)))));
          } else {
            kf = erff(xs) / (s2 * s) - sp * expf(-xs * xs) / s2;
          }
          if (QUAD) {
            if (xs < 1.f) {
              b2 = d2c * erf_series_2(x2);
              b3 = d3c * erf_series_3(x2);
            } else {
              const float e = expf(-x2), is2 = 1.f / s2;
              b2 = __builtin_fmaf(k2, e, -3.f * kf) * is2;
              b3 = __builtin_fmaf(k3, e, 5.f * b2) * is2;
            }
          }
        } else {
          const float e = expf(-xs * xs);
          kf = -(erfcf(xs) / (s2 * s) + sp * e / s2);
          if (QUAD) {
            const float is2 = 1.f / s2;
            b2 = __builtin_fmaf(k2, e, -3.f * kf) * is2;
            b3 = __builtin_fmaf(k3, e, 5.f * b2) * is2;
          }
        }
        ax = __builtin_fmaf(kf, sx, ax);
        ay = __builtin_fmaf(kf, sy, ay);
        az = __builtin_fmaf(kf, sz, az);
        if (QUAD) {
          const float Sx = a.GS[0] * sx + a.GS[3] * sy + a.GS[4] * sz;
          const float Sy = a.GS[3] * sx + a.GS[1] * sy + a.GS[5] * sz;
          const float Sz = a.GS[4] * sx + a.GS[5] * sy + a.GS[2] * sz;
          const float sSs = sx * Sx + sy * Sy + sz * Sz;
          const float cs = 0.5f * (tr * b2 - sSs * b3);
          qx += cs * sx + b2 * Sx;
          qy += cs * sy + b2 * Sy;
          qz += cs * sz + b2 * Sz;
        }
      }
  float bx = 0.f, by = 0.f, bz = 0.f;
  const float tx = r[0] * a.inv_L, ty = r[1] * a.inv_L, tz = r[2] * a.inv_L;
  for (int j = 0; j < nh; ++j) {
    const float4 h = htab[j];
    const float t = __builtin_fmaf(h.z, tz, __builtin_fmaf(h.y, ty, h.x * tx));
    const float w = h.w * sinpif(2.f * t);
    bx = __builtin_fmaf(w, h.x, bx);
    by = __builtin_fmaf(w, h.y, by);
    bz = __builtin_fmaf(w, h.z, bz);
  }
  float4* dst = a.acc + id;
  const float4 o = dev::gld(dst);
  if (QUAD) {
    bx += qx;
    by += qy;
    bz += qz;
  }
  dev::gst(dst, make_float4(o.x + a.GM * ax + bx, o.y + a.GM * ay + by, o.z + a.GM * az + bz, o.w));
}

}  // namespace

hipError_t launch_ewald(const EwaldArgs& a, hipStream_t s) {
  if (a.n_targets <= 0 || a.n_tasks <= 0) return hipSuccess;
  const int64_t g = (a.n_targets + kEwThreads - 1) / kEwThreads;
  if (a.quad) hipLaunchKernelGGL(k_ewald<true>, dim3((unsigned)g), dim3(kEwThreads), 0, s, a);
  else hipLaunchKernelGGL(k_ewald<false>, dim3((unsigned)g), dim3(kEwThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace gc
