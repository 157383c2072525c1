// Combined Lennard-Jones kernel over cell-pair tasks (Sec. 4.2: a compute
// object takes the particles of two patches and updates the forces of both).
//
// One wavefront per task.  Lanes are (i atom) x (j slice) as in the gravity
// kernel.  The j cell is staged in LDS with its image shift applied; forces
// on j atoms are accumulated in LDS with LDS float atomics, forces on i atoms
// in registers; at the end both are added to the global force array with one
// hardware FP32 atomic per atom component per task (a cell takes part in 14
// tasks as i and 13 as j).  A finishing kernel divides by the mass.
//
// Cutoff decision in FP32: per component d = (x_i - max(s,0)) - (x_j + min(s,0))
// (both inner operations are exact for wrapped coordinates, so d carries one
// rounding), r^2 = fma(dz, dz, fma(dy, dy, dx*dx)), inside iff r^2 < rc^2.
#include "gc_internal.h"

namespace gc {
namespace {

constexpr int kMaxTypes = 8;
constexpr int kLJTile = 128;  // j atoms per LDS tile

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
  int iter = 0;
  while (true) {
    // Persistent schedule: wave k of the grid starts with order[k], later tasks come from a
    // device counter offset by the number of waves in the grid.
    int got;
    if (PERSIST) {
      if (iter == 0) {
        got = uniform(blockIdx.x * wpb + wid);
      } else {
        int q = 0;
        if (lane == 0) q = atomicAdd(a.queue, 1);
        got = uniform(__shfl(q, 0, 64)) + (int)gridDim.x * wpb;
      }
      ++iter;
    } else {
      if (iter++) break;
      got = uniform(blockIdx.x * wpb + wid);
    }
    if (got >= a.n_tasks) break;
    const int t = PERSIST ? uniform(a.order[got]) : got;
    const gc_task tk = a.tasks[t];
    const int2 gj = a.ranges[tk.j_first];
    const int2 gjid = a.ranges_id[tk.j_first];
    const bool self = (tk.flags & GC_TASK_SELF) != 0;
    const float sa0 = tk.shift[0] > 0.f ? tk.shift[0] : 0.f, sb0 = tk.shift[0] < 0.f ? tk.shift[0] : 0.f;
    const float sa1 = tk.shift[1] > 0.f ? tk.shift[1] : 0.f, sb1 = tk.shift[1] < 0.f ? tk.shift[1] : 0.f;
    const float sa2 = tk.shift[2] > 0.f ? tk.shift[2] : 0.f, sb2 = tk.shift[2] < 0.f ? tk.shift[2] : 0.f;
    const int ipos0 = a.ibeg ? a.ibeg[t] : tk.i_begin;
    for (int i0 = 0; i0 < tk.i_count; i0 += 64) {
      const int icc = tk.i_count - i0 < 64 ? tk.i_count - i0 : 64;
      const int S = 64 / icc;
      const int il = lane % icc, sl = lane / icc;
      const bool active = sl < S;
      float xi = 0.f, yi = 0.f, zi = 0.f;
      int ti = 0;
      if (active) {
        float4 r = a.rec[ipos0 + i0 + il];
        xi = r.x - sa0; yi = r.y - sa1; zi = r.z - sa2;
        ti = (int)r.w;
      }
      float Fx = 0.f, Fy = 0.f, Fz = 0.f;
      for (int j0 = 0; j0 < gj.y; j0 += kLJTile) {
        const int cnt = gj.y - j0 < kLJTile ? gj.y - j0 : kLJTile;
        for (int e = lane; e < cnt; e += 64) {
          float4 r = a.rec[gj.x + j0 + e];
          jt[wid][e] = make_float4(r.x + sb0, r.y + sb1, r.z + sb2, r.w);
          fj[wid][0][e] = 0.f;
          fj[wid][1][e] = 0.f;
          fj[wid][2][e] = 0.f;
        }
        wave_sync();
        if (active) {
          const int C = (cnt + S - 1) / S;
          const int e0 = sl * C, e1 = e0 + C < cnt ? e0 + C : cnt;
          for (int e = e0; e < e1; ++e) {
            if (self && j0 + e <= i0 + il) continue;
            float4 j = jt[wid][e];
            float dx = xi - j.x, dy = yi - j.y, dz = zi - j.z;
            float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            if (r2 < a.rc2) {
              float2 p = tab[ti * a.n_types + (int)j.w];
              float ri2 = __builtin_amdgcn_rcpf(r2);
              float q = p.y * ri2;
              float q3 = q * q * q;
              float f = p.x * q3 * __builtin_fmaf(2.f, q3, -1.f) * ri2;
              Fx = __builtin_fmaf(f, dx, Fx);
              Fy = __builtin_fmaf(f, dy, Fy);
              Fz = __builtin_fmaf(f, dz, Fz);
              atomicAdd(&fj[wid][0][e], -f * dx);
              atomicAdd(&fj[wid][1][e], -f * dy);
              atomicAdd(&fj[wid][2][e], -f * dz);
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
      // reduce the slices of each i atom
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
        float4* dst = a.acc + (tk.i_begin + i0 + lane);
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
  if (a.n_tasks <= 0) return hipSuccess;
  (void)wpb;
  if (persistent) {
    hipLaunchKernelGGL(k_lj<true>, dim3(grid), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_lj<false>, dim3((a.n_tasks + 3) / 4), dim3(256), 0, s, a);
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
