// Combined Barnes-Hut force kernel, one launch per batch: one workgroup per
// task (task order longest first), or a persistent grid that takes tasks from
// a device counter.  The per-task code is in grav_dev.h.
#include "grav_dev.h"

namespace gc {
namespace {

using dev::grav_lds_per_wave;
using dev::grav_task;
using dev::uniform;

// Tasks a persistent block takes per grab of the shared counter (consecutive tasks of the
// longest-first order have similar costs, so a grab of a few keeps the blocks balanced while the
// counter, one address for the whole grid, sees a few times fewer atomics).
constexpr int kGrabTasks = 4;

template <int ORDER, bool LISTS, bool PERSIST, int TPL, bool POT = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) k_grav(GravArgs a) {
  extern __shared__ float4 smem[];
  __shared__ int s_task;
  int iter = 0;
  int chunk = 0, left = 0;
  while (true) {
    // Tasks run in longest-first order: block b starts with order[b]; in the persistent
    // schedule block b first takes tasks [b k, b k + k) (k = kGrabTasks) and later grabs of k come
    // from a device counter (offset by the grid's first grabs), so the first grabs need no atomics.
    int got;
    if (PERSIST) {
      if (left == 0) {
        if (iter == 0) {
          chunk = (int)blockIdx.x * kGrabTasks;
        } else {
          if (threadIdx.x == 0) s_task = (int)gridDim.x * kGrabTasks + atomicAdd(a.queue, kGrabTasks);
          __syncthreads();
          chunk = uniform(s_task);
          __syncthreads();
        }
        left = kGrabTasks;
      }
      got = chunk + (kGrabTasks - left);
      --left;
      ++iter;
    } else {
      if (iter++) break;
      got = blockIdx.x;
    }
    if (got >= a.n_tasks) break;
    const int t = uniform(a.order[got]);
    const gc_task g = a.tasks[t];
    const dev::TaskDesc td{uniform(g.i_begin), uniform(g.i_count), uniform(g.j_first), uniform(g.j_nranges),
                           uniform(g.n_first), uniform(g.n_count), uniform(a.ibeg ? a.ibeg[t] : g.i_begin)};
    dev::NodePrefetch<ORDER> pf;
    grav_task<ORDER, LISTS, TPL, POT>(a, t, td, smem, pf, false, [] {}, [](int) {});
  }
}

template <int ORDER, bool LISTS, bool PERSIST, int TPL>
hipError_t launch_one(const GravArgs& a, int wpb, int grid, hipStream_t s) {
  size_t lds = (size_t)wpb * grav_lds_per_wave(a.tile) * sizeof(float4);
  if (!PERSIST) grid = a.n_tasks;
  if (grid < 1) return hipSuccess;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, LISTS, PERSIST, TPL>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grav<ORDER, LISTS, PERSIST, TPL>), dim3(grid), dim3(64 * wpb), lds, s, a);
  return hipGetLastError();
}

template <int ORDER, bool LISTS, bool PERSIST, int TPL>
hipError_t occ_one(int tile, int wpb, int* blocks) {
  size_t lds = (size_t)wpb * grav_lds_per_wave(tile) * sizeof(float4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, LISTS, PERSIST, TPL>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_grav<ORDER, LISTS, PERSIST, TPL>, 64 * wpb, lds);
}

template <int ORDER, bool LISTS, bool PERSIST>
hipError_t launch_two(int tpl, const GravArgs& a, int wpb, int grid, hipStream_t s) {
  if (tpl == 2) return launch_one<ORDER, LISTS, PERSIST, 2>(a, wpb, grid, s);
  if (tpl == 3) return launch_one<ORDER, LISTS, PERSIST, 3>(a, wpb, grid, s);
  return launch_one<ORDER, LISTS, PERSIST, 1>(a, wpb, grid, s);
}

template <int ORDER, bool LISTS, bool PERSIST>
hipError_t occ_two(int tpl, int tile, int wpb, int* blocks) {
  if (tpl == 2) return occ_one<ORDER, LISTS, PERSIST, 2>(tile, wpb, blocks);
  if (tpl == 3) return occ_one<ORDER, LISTS, PERSIST, 3>(tile, wpb, blocks);
  return occ_one<ORDER, LISTS, PERSIST, 1>(tile, wpb, blocks);
}

// Per-round arguments read through the constant address space: with a uniform index they come in by
// scalar loads into scalar registers.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cst(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}
template <class T>
__device__ __forceinline__ T cload(const __attribute__((address_space(4))) T* p) {
  static_assert(sizeof(T) % 4 == 0, "word copy");
  T v;
  const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)p;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return v;
}

// Every task of several rounds in one launch: block b runs item b (its round's index in `kind`, its
// task's fields and first packed target), with that round's arguments.
template <int ORDER, int TPL>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
    k_grav_rounds(const StepItem* __restrict__ items, const GravArgs* __restrict__ rounds) {
  extern __shared__ float4 smem[];
  const StepItem it = cload(&cst(items)[blockIdx.x]);
  const GravArgs ga = cload(&cst(rounds)[it.kind]);
  const dev::TaskDesc td{it.i_begin, it.i_count, it.j_first, it.j_nranges, it.n_first, it.n_count, it.idx};
  dev::NodePrefetch<ORDER> pf;
  grav_task<ORDER, false, TPL>(ga, 0, td, smem, pf, false, [] {}, [](int) {});
}

template <int ORDER, int TPL>
hipError_t launch_rounds_one(const StepItem* items, int32_t n_items, const GravArgs* rounds, int tile, int wpb,
                             hipStream_t s) {
  const size_t lds = (size_t)wpb * grav_lds_per_wave(tile) * sizeof(float4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav_rounds<ORDER, TPL>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grav_rounds<ORDER, TPL>), dim3(n_items), dim3(64 * wpb), lds, s, items, rounds);
  return hipGetLastError();
}

// The potential variant: one workgroup per task, one target per lane, records in position space.
template <int ORDER>
hipError_t launch_pot(const GravArgs& a, int wpb, hipStream_t s) {
  const size_t lds = (size_t)wpb * grav_lds_per_wave(a.tile, true) * sizeof(float4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, false, false, 1, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grav<ORDER, false, false, 1, true>), dim3(a.n_tasks), dim3(64 * wpb), lds, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grav_rounds(int order, int tpl, const StepItem* items, int32_t n_items, const GravArgs* rounds,
                              int tile, int wpb, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (order == 1) {
    if (tpl == 2) return launch_rounds_one<1, 2>(items, n_items, rounds, tile, wpb, s);
    if (tpl == 3) return launch_rounds_one<1, 3>(items, n_items, rounds, tile, wpb, s);
    return launch_rounds_one<1, 1>(items, n_items, rounds, tile, wpb, s);
  }
  if (tpl == 2) return launch_rounds_one<2, 2>(items, n_items, rounds, tile, wpb, s);
  if (tpl == 3) return launch_rounds_one<2, 3>(items, n_items, rounds, tile, wpb, s);
  return launch_rounds_one<2, 1>(items, n_items, rounds, tile, wpb, s);
}

hipError_t launch_grav_potential(int order, const GravArgs& a, int wpb, hipStream_t s) {
  if (a.n_tasks <= 0) return hipSuccess;
  return order == 1 ? launch_pot<1>(a, wpb, s) : launch_pot<2>(a, wpb, s);
}

hipError_t launch_grav(int order, bool lists, bool persistent, int tpl, const GravArgs& a, int wpb, int grid,
                       hipStream_t s) {
  if (a.n_tasks <= 0) return hipSuccess;
  if (order == 1) {
    if (lists) return persistent ? launch_two<1, true, true>(tpl, a, wpb, grid, s) : launch_two<1, true, false>(tpl, a, wpb, grid, s);
    return persistent ? launch_two<1, false, true>(tpl, a, wpb, grid, s) : launch_two<1, false, false>(tpl, a, wpb, grid, s);
  }
  if (lists) return persistent ? launch_two<2, true, true>(tpl, a, wpb, grid, s) : launch_two<2, true, false>(tpl, a, wpb, grid, s);
  return persistent ? launch_two<2, false, true>(tpl, a, wpb, grid, s) : launch_two<2, false, false>(tpl, a, wpb, grid, s);
}

hipError_t grav_occupancy(int order, bool lists, bool persistent, int tpl, int tile, int wpb, int* blocks) {
  if (order == 1) {
    if (lists) return persistent ? occ_two<1, true, true>(tpl, tile, wpb, blocks) : occ_two<1, true, false>(tpl, tile, wpb, blocks);
    return persistent ? occ_two<1, false, true>(tpl, tile, wpb, blocks) : occ_two<1, false, false>(tpl, tile, wpb, blocks);
  }
  if (lists) return persistent ? occ_two<2, true, true>(tpl, tile, wpb, blocks) : occ_two<2, true, false>(tpl, tile, wpb, blocks);
  return persistent ? occ_two<2, false, true>(tpl, tile, wpb, blocks) : occ_two<2, false, false>(tpl, tile, wpb, blocks);
}

}  // namespace gc
