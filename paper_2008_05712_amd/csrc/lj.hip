// Combined Lennard-Jones kernel over cell-pair tasks (Sec. 4.2: a compute
// object takes the particles of two patches and updates the forces of both).
//
// One wavefront per run of consecutive tasks that share one target range (a
// cell's self task and its 13 half-shell neighbours form one run), so the
// i-side forces stay in registers across the run and reach memory once.
// Lanes are (i atom) x (j slice) as in the gravity kernel.  Each j cell is
// staged in LDS with its image shift applied; j-side forces accumulate in LDS
// with LDS float atomics, and the lanes of a slice walk its j entries with a
// per-lane rotation so they touch different entries at each step.  Both sides
// reach the global force array through hardware FP32 atomics; a finishing
// kernel divides by the mass.
//
// Cutoff decision in FP32: per component d = (x_i - max(s,0)) - (x_j + min(s,0))
// (both inner operations are exact for wrapped coordinates, so d carries one
// rounding), r^2 = fma(dz, dz, fma(dy, dy, dx*dx)), inside iff r^2 < rc^2.
#include "gc_internal.h"

namespace gc {
namespace {

constexpr int kMaxTypes = 8;
constexpr int kLJTile = 128;  // j atoms per LDS tile
constexpr int kRunChunk = 16; // runs per grab in the persistent schedule

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <bool PERSIST>
__global__ void __launch_bounds__(256) k_lj(LJArgs a) {
  __shared__ float2 tab[kMaxTypes * kMaxTypes];              // (24 eps_ij, sigma_ij^2)
  __shared__ float4 jt[4][kLJTile];                          // j records, shifted
  __shared__ float fj[4][3][kLJTile];                        // j force accumulators
  __shared__ float fi[4][3][64];
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int wpb = blockDim.x >> 6;
  for (int k = threadIdx.x; k < a.n_types * a.n_types; k += blockDim.x) {
    int ta = k / a.n_types, tb = k % a.n_types;
    float e = sqrtf(a.eps_t[ta] * a.eps_t[tb]);
    float sg = 0.5f * (a.sig_t[ta] + a.sig_t[tb]);
    tab[k] = make_float2(24.f * e, sg * sg);
  }
  __syncthreads();
  // persistent: wave k takes runs [k * chunk, k * chunk + chunk), then chunks from a counter
  // (chunk starts only grow, so the first run past the end ends the wave)
  int chunk_base = uniform((blockIdx.x * wpb + wid) * (PERSIST ? kRunChunk : 1));
  int chunk_left = PERSIST ? kRunChunk : 1;
  while (true) {
    if (chunk_left == 0) {
      if (!PERSIST) break;
      int q = 0;
      if (lane == 0) q = atomicAdd(a.queue, 1);
      chunk_base = uniform((__shfl(q, 0, 64) + (int)gridDim.x * wpb) * kRunChunk);
      chunk_left = kRunChunk;
    }
    const int r = chunk_base + (PERSIST ? kRunChunk - chunk_left : 0);
    --chunk_left;
    if (r >= a.n_runs) break;
    const int t0 = uniform(a.runs[r]), t1 = uniform(a.runs[r + 1]);
    const gc_task tk0 = a.tasks[t0];
    const int ipos0 = a.ibeg ? a.ibeg[t0] : tk0.i_begin;
    for (int i0 = 0; i0 < tk0.i_count; i0 += 64) {
      const int icc = tk0.i_count - i0 < 64 ? tk0.i_count - i0 : 64;
      const int S = 64 / icc;
      const int il = lane % icc, sl = lane / icc;
      const bool active = sl < S;
      float xr = 0.f, yr = 0.f, zr = 0.f;
      int ti = 0;
      if (active) {
        float4 rr = a.rec[ipos0 + i0 + il];
        xr = rr.x; yr = rr.y; zr = rr.z;
        ti = (int)rr.w;
      }
      float Fx = 0.f, Fy = 0.f, Fz = 0.f;
      for (int t = t0; t < t1; ++t) {
        const gc_task tk = a.tasks[t];
        const int2 gj = a.ranges[tk.j_first];
        const int2 gjid = a.ranges_id[tk.j_first];
        const bool self = (tk.flags & GC_TASK_SELF) != 0;
        const float xi = xr - (tk.shift[0] > 0.f ? tk.shift[0] : 0.f);
        const float yi = yr - (tk.shift[1] > 0.f ? tk.shift[1] : 0.f);
        const float zi = zr - (tk.shift[2] > 0.f ? tk.shift[2] : 0.f);
        const float sb0 = tk.shift[0] < 0.f ? tk.shift[0] : 0.f;
        const float sb1 = tk.shift[1] < 0.f ? tk.shift[1] : 0.f;
        const float sb2 = tk.shift[2] < 0.f ? tk.shift[2] : 0.f;
        for (int j0 = 0; j0 < gj.y; j0 += kLJTile) {
          const int cnt = gj.y - j0 < kLJTile ? gj.y - j0 : kLJTile;
          for (int e = lane; e < cnt; e += 64) {
            float4 rj = a.rec[gj.x + j0 + e];
            jt[wid][e] = make_float4(rj.x + sb0, rj.y + sb1, rj.z + sb2, rj.w);
            fj[wid][0][e] = 0.f;
            fj[wid][1][e] = 0.f;
            fj[wid][2][e] = 0.f;
          }
          wave_sync();
          if (active) {
            const int C = (cnt + S - 1) / S;
            const int e0 = sl * C, e1 = e0 + C < cnt ? e0 + C : cnt;
            const int cs = e1 - e0;
            if (cs > 0) {
              int e = e0 + il % cs;  // lanes of a slice start at different entries
              for (int k = 0; k < cs; ++k) {
                if (!(self && j0 + e <= i0 + il)) {
                  const float4 j = jt[wid][e];
                  const float dx = xi - j.x, dy = yi - j.y, dz = zi - j.z;
                  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                  if (r2 < a.rc2) {
                    const float2 p = tab[ti * a.n_types + (int)j.w];
                    const float ri2 = __builtin_amdgcn_rcpf(r2);
                    const float q = p.y * ri2;
                    const float q3 = q * q * q;
                    const float f = p.x * q3 * __builtin_fmaf(2.f, q3, -1.f) * ri2;
                    Fx = __builtin_fmaf(f, dx, Fx);
                    Fy = __builtin_fmaf(f, dy, Fy);
                    Fz = __builtin_fmaf(f, dz, Fz);
                    atomicAdd(&fj[wid][0][e], -f * dx);
                    atomicAdd(&fj[wid][1][e], -f * dy);
                    atomicAdd(&fj[wid][2][e], -f * dz);
                  }
                }
                e = (e + 1 == e1) ? e0 : e + 1;
              }
            }
          }
          wave_sync();
          for (int e = lane; e < cnt; e += 64) {
            float4* dst = a.acc + (gjid.x + j0 + e);
            unsafeAtomicAdd(&dst->x, fj[wid][0][e]);
            unsafeAtomicAdd(&dst->y, fj[wid][1][e]);
            unsafeAtomicAdd(&dst->z, fj[wid][2][e]);
          }
          wave_sync();
        }
      }
      // reduce the slices of each i atom over the whole run, one atomic per component
      fi[wid][0][lane] = Fx;
      fi[wid][1][lane] = Fy;
      fi[wid][2][lane] = Fz;
      wave_sync();
      if (lane < icc) {
        float sx = 0.f, sy = 0.f, sz = 0.f;
        for (int s = 0; s < S; ++s) {
          sx += fi[wid][0][s * icc + lane];
          sy += fi[wid][1][s * icc + lane];
          sz += fi[wid][2][s * icc + lane];
        }
        float4* dst = a.acc + (tk0.i_begin + i0 + lane);
        unsafeAtomicAdd(&dst->x, sx);
        unsafeAtomicAdd(&dst->y, sy);
        unsafeAtomicAdd(&dst->z, sz);
      }
      wave_sync();
    }
  }
}

__global__ void k_lj_finish(float4* __restrict__ acc, const float* __restrict__ mass_t,
                            const float4* __restrict__ rec_by_id, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float4 f = acc[i];
    float m = mass_t[(int)rec_by_id[i].w];
    acc[i] = make_float4(f.x / m, f.y / m, f.z / m, 0.f);
  }
}

}  // namespace

hipError_t launch_lj(bool persistent, const LJArgs& a, int wpb, int grid, hipStream_t s) {
  if (a.n_runs <= 0) return hipSuccess;
  (void)wpb;
  if (persistent) {
    int g = grid;
    const int need = (a.n_runs + 4 * kRunChunk - 1) / (4 * kRunChunk);
    if (g > need) g = need;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_lj<true>, dim3(g), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_lj<false>, dim3((a.n_runs + 3) / 4), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_lj_finish(float4* acc, const float* mass_t, const float4* rec_by_id, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_lj_finish, dim3(g), dim3(256), 0, s, acc, mass_t, rec_by_id, n);
  return hipGetLastError();
}

}  // namespace gc
