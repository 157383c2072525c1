// Combined Lennard-Jones kernels over cell-pair tasks (Sec. 4.2: a compute
// object takes the particles of two patches and updates the forces of both).
// Two forms: the gather form further below, used whenever the batch's target
// ranges are equal or disjoint (cell tasks always are), and the half-shell form
// described here, for any other task set.
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
#include "grav_dev.h"
#include "mem_dev.h"

namespace gc {
namespace {

using dev::gld;
using dev::gst;

constexpr int kMaxTypes = 8;
constexpr int kLJTile = 128;  // j atoms per LDS tile
constexpr int kRunChunk = 16; // runs per grab in the persistent schedule

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

// ---------------------------------------------------------------- gather form
//
// One wavefront per target range (a cell): every task that has the cell on either side contributes
// to its atoms, so each pair of two different cells is evaluated once from each side (the self task
// of a cell once, from all its atoms).  The cell's atoms sum their forces in registers and each
// atom's acceleration is written once: no atomics, the same bits on every run and schedule.  Work
// per pair doubles against the half-shell form above, but a pair costs about 20 VALU operations
// there and the atomics, per-task waits and LDS atomics of the half-shell form cost more.
//
// A wavefront stages the sources of up to 32 tasks at a time in LDS tiles (shifted as below) and
// splits its 64 lanes into (target atom) x (source slice) as the gravity kernel does; the slices
// are reduced through LDS at the end.  The cutoff decision takes the same FP32 operations as the
// half-shell form, from either side: for a task with shift s, a = max(s, 0), b = min(s, 0), the
// separation is d = (x_i - a) - (x_j + b); the task's i atom as target gets F += f d, its j atom
// gets F += f (-d), computed as (x_j + b) - (x_i - a), the exact negation, so r^2 is the same.
// The per-task shift sits on the source when staged (x_j + b, or x_i + (-a)); on the target side
// it is added per pair, only in cells that have tasks across the periodic boundary (x + (-a) and
// x - a round alike).  A zero separation is the atom itself (a cell's self task) and adds nothing.
//
// Candidates are pruned as they are staged: a source whose distance from the bounding box of the
// wavefront's target atoms (in the targets' frame, the source's position less its task's target
// shift) exceeds r_c is within r_c of none of them and is left out; the survivors of each staged
// group of up to 64 sources are compacted into the tile in their order.  The test keeps a source
// up to (1 + 1e-3) r_c^2 from the box, far beyond FP32 rounding, so no pair that the cutoff
// decision accepts is dropped; the decision itself is unchanged.
constexpr int kGTile = 64;   // source records per LDS tile per wavefront
constexpr int kEGroup = 32;  // tasks whose sources a wavefront stages at a time
constexpr float kFar = 1e18f;  // padding sources: r^2 ~ 3e36, finite and outside any cutoff

template <bool SHIFTED, bool ONE>
__device__ __forceinline__ void gather_tile(const float4* __restrict__ p, const float4* __restrict__ o, int C,
                                            float tx, float ty, float tz, const float2* __restrict__ trow,
                                            float2 p0, float rc2, float& Fx, float& Fy, float& Fz) {
#pragma unroll 2
  for (int k = 0; k < C; ++k) {
    const float4 sj = p[k];
    float ux = tx, uy = ty, uz = tz;
    if (SHIFTED) {
      const float4 w = o[k];
      ux = tx + w.x;
      uy = ty + w.y;
      uz = tz + w.z;
    }
    const float ex = ux - sj.x, ey = uy - sj.y, ez = uz - sj.z;
    const float r2 = __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex));
    const float2 pp = ONE ? p0 : trow[(int)sj.w];
    const float ri2 = __builtin_amdgcn_rcpf(r2);
    const float q = pp.y * ri2;
    const float q3 = q * q * q;
    float f = pp.x * q3 * __builtin_fmaf(2.f, q3, -1.f) * ri2;
    f = (r2 < rc2 && r2 > 0.f) ? f : 0.f;
    Fx = __builtin_fmaf(f, ex, Fx);
    Fy = __builtin_fmaf(f, ey, Fy);
    Fz = __builtin_fmaf(f, ez, Fz);
  }
}

template <bool PERSIST, bool ONE>
__global__ void __launch_bounds__(256) k_lj_gather(LJArgs a) {
  __shared__ float2 tab[kMaxTypes * kMaxTypes];  // (24 eps_ij, sigma_ij^2)
  __shared__ float4 src[4][kGTile];              // sources, shifted; padding far away
  __shared__ float4 tof[4][kGTile];              // per source: its task's target-side shift
  __shared__ float4 esh[4][kEGroup], eto[4][kEGroup];  // per task of the group: source and target shifts
  __shared__ int eoff[4][kEGroup], ebeg[4][kEGroup];   // per task: first flat source, first source record
  __shared__ float fr[4][3][64];
  const int lane = threadIdx.x & 63;
  const int wid = uniform(threadIdx.x >> 6);
  const int wpb = blockDim.x >> 6;
  for (int k = threadIdx.x; k < a.n_types * a.n_types; k += blockDim.x) {
    const int ta = k / a.n_types, tb = k % a.n_types;
    const float e = sqrtf(a.eps_t[ta] * a.eps_t[tb]);
    const float sg = 0.5f * (a.sig_t[ta] + a.sig_t[tb]);
    tab[k] = make_float2(24.f * e, sg * sg);
  }
  __syncthreads();
  const float2 p0 = tab[0];
  const int32_t* tw0 = reinterpret_cast<const int32_t*>(a.tasks);
  constexpr int kTaskWords = sizeof(gc_task) / 4;
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
    const int g = chunk_base + (PERSIST ? kRunChunk - chunk_left : 0);
    --chunk_left;
    if (g >= a.n_tgt) break;
    const int4 tg = gld(a.tgt + g);  // (first id, count, first entry, entries)
    const int id0 = uniform(tg.x), cnt = uniform(tg.y), e0 = uniform(tg.z), ne = uniform(tg.w);
    // the range's first record, from its first entry
    const int en0 = uniform(gld(a.ent + e0));
    const int32_t* tw = tw0 + (int64_t)(en0 >> 1) * kTaskWords;
    const int rb = (en0 & 1) ? uniform(gld(a.ranges + uniform(gld(tw + 2))).x)
                             : (a.ibeg ? uniform(gld(a.ibeg + (en0 >> 1))) : uniform(gld(tw)));
    for (int i0 = 0; i0 < cnt; i0 += 64) {
      const int icc = cnt - i0 < 64 ? cnt - i0 : 64;
      const int S = 64 / icc;
      const int il = lane % icc, sl = lane / icc;
      const bool active = sl < S;
      float tx = 0.f, ty = 0.f, tz = 0.f;
      int ti = 0;
      if (active) {
        const float4 r = gld(a.rec + rb + i0 + il);
        tx = r.x; ty = r.y; tz = r.z;
        ti = (int)r.w;
      }
      const float2* trow = tab + ti * a.n_types;
      float Fx = 0.f, Fy = 0.f, Fz = 0.f;
      const int DT = S * (kGTile / S);
      // the targets' bounding box (lanes without a target are neutral)
      const float blx = wave_min(active ? tx : kFar), bly = wave_min(active ? ty : kFar),
                  blz = wave_min(active ? tz : kFar);
      const float bhx = wave_max(active ? tx : -kFar), bhy = wave_max(active ? ty : -kFar),
                  bhz = wave_max(active ? tz : -kFar);
      const float keep2 = a.rc2 * 1.001f;
      for (int eg = 0; eg < ne; eg += kEGroup) {
        const int nen = ne - eg < kEGroup ? ne - eg : kEGroup;
        int n = 0, sb = 0;
        float4 sh = make_float4(0.f, 0.f, 0.f, 0.f), to = sh;
        if (lane < nen) {
          const int en = gld(a.ent + e0 + eg + lane);
          const int t = en >> 1;
          const int32_t* w = tw0 + (int64_t)t * kTaskWords;
          const float s0 = __int_as_float(gld(w + 7)), s1 = __int_as_float(gld(w + 8)),
                      s2 = __int_as_float(gld(w + 9));
          const float ax = s0 > 0.f ? s0 : 0.f, ay = s1 > 0.f ? s1 : 0.f, az = s2 > 0.f ? s2 : 0.f;
          const float bx = s0 < 0.f ? s0 : 0.f, by = s1 < 0.f ? s1 : 0.f, bz = s2 < 0.f ? s2 : 0.f;
          if (en & 1) {  // target on the task's j side: sources are its i atoms, x_i - a
            sb = a.ibeg ? gld(a.ibeg + t) : gld(w);
            n = gld(w + 1);
            sh = make_float4(-ax, -ay, -az, 0.f);
            to = make_float4(bx, by, bz, 0.f);
          } else {       // target on the task's i side: sources are its j atoms, x_j + b
            const int2 jr = gld(a.ranges + gld(w + 2));
            sb = jr.x;
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
          esh[wid][lane] = sh;
          eto[wid][lane] = to;
        }
        wave_sync();
        for (int ws = 0; ws < total; ws += DT) {
          // one source per lane (DT <= 64): staged, tested, and the survivors compacted
          const int c = total - ws < DT ? total - ws : DT;
          float4 v = make_float4(kFar, kFar, kFar, 0.f), o = make_float4(0.f, 0.f, 0.f, 0.f);
          bool keep = false;
          if (lane < c) {
            const int f = ws + lane;
            int lo = 0, hi = nen - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (eoff[wid][mid] <= f) lo = mid;
              else hi = mid - 1;
            }
            const float4 r = gld(a.rec + ebeg[wid][lo] + (f - eoff[wid][lo]));
            const float4 q = esh[wid][lo];
            v = make_float4(r.x + q.x, r.y + q.y, r.z + q.z, r.w);
            o = eto[wid][lo];
            const float px = v.x - o.x, py = v.y - o.y, pz = v.z - o.z;
            const float dx = fmaxf(fmaxf(blx - px, px - bhx), 0.f);
            const float dy = fmaxf(fmaxf(bly - py, py - bhy), 0.f);
            const float dz = fmaxf(fmaxf(blz - pz, pz - bhz), 0.f);
            keep = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)) <= keep2;
          }
          const uint64_t km = __ballot(keep);
          const int kc = uniform(__popcll(km));
          const int C = (kc + S - 1) / S;
          const int padded = S * C;
          if (keep) {
            const int k = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
            src[wid][k] = v;
            if (shifted) tof[wid][k] = o;
          }
          if (lane >= kc && lane < padded) {
            src[wid][lane] = make_float4(kFar, kFar, kFar, 0.f);
            if (shifted) tof[wid][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
          wave_sync();
          if (active && C > 0) {
            if (shifted)
              gather_tile<true, ONE>(&src[wid][sl * C], &tof[wid][sl * C], C, tx, ty, tz, trow, p0, a.rc2, Fx, Fy, Fz);
            else
              gather_tile<false, ONE>(&src[wid][sl * C], nullptr, C, tx, ty, tz, trow, p0, a.rc2, Fx, Fy, Fz);
          }
          wave_sync();
        }
      }
      // the slices of each target atom, in a fixed order; a = F / m
      fr[wid][0][lane] = Fx;
      fr[wid][1][lane] = Fy;
      fr[wid][2][lane] = Fz;
      wave_sync();
      if (lane < icc) {
        float sx = 0.f, sy = 0.f, sz = 0.f;
        for (int s = 0; s < S; ++s) {
          sx += fr[wid][0][s * icc + lane];
          sy += fr[wid][1][s * icc + lane];
          sz += fr[wid][2][s * icc + lane];
        }
        const float m = a.mass_t[ti];
        gst(a.acc + id0 + i0 + lane, make_float4(sx / m, sy / m, sz / m, 0.f));
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

// In-cutoff pairs of the tasks (self tasks: i < j), with the forward kernels' FP32 decision: one
// wavefront per task at a time, lanes over the task's flattened (i, j) candidates.
__global__ void __launch_bounds__(256) k_lj_count(const gc_task* __restrict__ tasks, int32_t n_tasks,
                                                  const int2* __restrict__ ranges_id,
                                                  const float4* __restrict__ rec_by_id, float rc2,
                                                  unsigned long long* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  unsigned long long cnt = 0;
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < n_tasks; t += (int64_t)gridDim.x * 4) {
    const gc_task tk = tasks[t];
    const int2 g = ranges_id[tk.j_first];
    const bool self = (tk.flags & GC_TASK_SELF) != 0;
    const float a0 = tk.shift[0] > 0.f ? tk.shift[0] : 0.f, b0 = tk.shift[0] < 0.f ? tk.shift[0] : 0.f;
    const float a1 = tk.shift[1] > 0.f ? tk.shift[1] : 0.f, b1 = tk.shift[1] < 0.f ? tk.shift[1] : 0.f;
    const float a2 = tk.shift[2] > 0.f ? tk.shift[2] : 0.f, b2 = tk.shift[2] < 0.f ? tk.shift[2] : 0.f;
    const int64_t np = (int64_t)max(tk.i_count, 0) * max(g.y, 0);
    for (int64_t p = lane; p < np; p += 64) {
      const int i = (int)(p / g.y), j = (int)(p - (int64_t)i * g.y);
      if (self && j <= i) continue;
      const float4 xi = rec_by_id[tk.i_begin + i], xj = rec_by_id[g.x + j];
      const float dx = (xi.x - a0) - (xj.x + b0);
      const float dy = (xi.y - a1) - (xj.y + b1);
      const float dz = (xi.z - a2) - (xj.z + b2);
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      cnt += r2 < rc2 ? 1ull : 0ull;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0 && cnt) atomicAdd(out, cnt);
}

}  // namespace

hipError_t launch_lj_count(const gc_task* tasks, int32_t n_tasks, const int2* ranges_id, const float4* rec_by_id,
                           float rc2, unsigned long long* out, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  int g = (n_tasks + 3) / 4;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_lj_count, dim3(g), dim3(256), 0, s, tasks, n_tasks, ranges_id, rec_by_id, rc2, out);
  return hipGetLastError();
}

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

hipError_t launch_lj_gather(bool persistent, const LJArgs& a, int grid, hipStream_t s) {
  if (a.n_tgt <= 0) return hipSuccess;
  const bool one = a.n_types == 1;
  if (persistent) {
    int g = grid;
    const int need = (a.n_tgt + 4 * kRunChunk - 1) / (4 * kRunChunk);
    if (g > need) g = need;
    if (g < 1) g = 1;
    if (one) hipLaunchKernelGGL((k_lj_gather<true, true>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_lj_gather<true, false>), dim3(g), dim3(256), 0, s, a);
  } else {
    const int g = (a.n_tgt + 3) / 4;
    if (one) hipLaunchKernelGGL((k_lj_gather<false, true>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_lj_gather<false, false>), dim3(g), dim3(256), 0, s, a);
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
