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

template <int ORDER, bool LISTS, bool PERSIST, bool TWO, bool POT = false>
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
    grav_task<ORDER, LISTS, TWO, POT>(a, t, td, smem, pf, false, [] {}, [](int) {});
  }
}

template <int ORDER, bool LISTS, bool PERSIST, bool TWO>
hipError_t launch_one(const GravArgs& a, int wpb, int grid, hipStream_t s) {
  size_t lds = (size_t)wpb * grav_lds_per_wave(a.tile) * sizeof(float4);
  if (!PERSIST) grid = a.n_tasks;
  if (grid < 1) return hipSuccess;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, LISTS, PERSIST, TWO>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grav<ORDER, LISTS, PERSIST, TWO>), dim3(grid), dim3(64 * wpb), lds, s, a);
  return hipGetLastError();
}

template <int ORDER, bool LISTS, bool PERSIST, bool TWO>
hipError_t occ_one(int tile, int wpb, int* blocks) {
  size_t lds = (size_t)wpb * grav_lds_per_wave(tile) * sizeof(float4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, LISTS, PERSIST, TWO>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_grav<ORDER, LISTS, PERSIST, TWO>, 64 * wpb, lds);
}

template <int ORDER, bool LISTS, bool PERSIST>
hipError_t launch_two(bool two, const GravArgs& a, int wpb, int grid, hipStream_t s) {
  return two ? launch_one<ORDER, LISTS, PERSIST, true>(a, wpb, grid, s)
             : launch_one<ORDER, LISTS, PERSIST, false>(a, wpb, grid, s);
}

template <int ORDER, bool LISTS, bool PERSIST>
hipError_t occ_two(bool two, int tile, int wpb, int* blocks) {
  return two ? occ_one<ORDER, LISTS, PERSIST, true>(tile, wpb, blocks)
             : occ_one<ORDER, LISTS, PERSIST, false>(tile, wpb, blocks);
}

// The potential variant: one workgroup per task, one target per lane, records in position space.
template <int ORDER>
hipError_t launch_pot(const GravArgs& a, int wpb, hipStream_t s) {
  const size_t lds = (size_t)wpb * grav_lds_per_wave(a.tile, true) * sizeof(float4);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_grav<ORDER, false, false, false, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_grav<ORDER, false, false, false, true>), dim3(a.n_tasks), dim3(64 * wpb), lds, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grav_potential(int order, const GravArgs& a, int wpb, hipStream_t s) {
  if (a.n_tasks <= 0) return hipSuccess;
  return order == 1 ? launch_pot<1>(a, wpb, s) : launch_pot<2>(a, wpb, s);
}

hipError_t launch_grav(int order, bool lists, bool persistent, bool two, const GravArgs& a, int wpb, int grid,
                       hipStream_t s) {
  if (a.n_tasks <= 0) return hipSuccess;
  if (order == 1) {
    if (lists) return persistent ? launch_two<1, true, true>(two, a, wpb, grid, s) : launch_two<1, true, false>(two, a, wpb, grid, s);
    return persistent ? launch_two<1, false, true>(two, a, wpb, grid, s) : launch_two<1, false, false>(two, a, wpb, grid, s);
  }
  if (lists) return persistent ? launch_two<2, true, true>(two, a, wpb, grid, s) : launch_two<2, true, false>(two, a, wpb, grid, s);
  return persistent ? launch_two<2, false, true>(two, a, wpb, grid, s) : launch_two<2, false, false>(two, a, wpb, grid, s);
}

hipError_t grav_occupancy(int order, bool lists, bool persistent, bool two, int tile, int wpb, int* blocks) {
  if (order == 1) {
    if (lists) return persistent ? occ_two<1, true, true>(two, tile, wpb, blocks) : occ_two<1, true, false>(two, tile, wpb, blocks);
    return persistent ? occ_two<1, false, true>(two, tile, wpb, blocks) : occ_two<1, false, false>(two, tile, wpb, blocks);
  }
  if (lists) return persistent ? occ_two<2, true, true>(two, tile, wpb, blocks) : occ_two<2, true, false>(two, tile, wpb, blocks);
  return persistent ? occ_two<2, false, true>(two, tile, wpb, blocks) : occ_two<2, false, false>(two, tile, wpb, blocks);
}

}  // namespace gc
