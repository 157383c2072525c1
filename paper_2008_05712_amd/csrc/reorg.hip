// Reorganisation kernels (Sec. 3.2): residency lookup of the combined
// request's union in the chare table, slot assignment and staging of missing
// records, the packing gather (or the source gather for redundant transfers),
// the address-list remaps, and eviction.
//
// The union U of a batch (sorted distinct ids over its target and direct
// ranges) and every position in it are fixed when the batch is committed: the
// host builds them once, as the runtime keeps its index lists sorted on
// insertion.  What depends on the pool's state is done here, in one launch:
//   k_reorg  blocks take tickets in dispatch order.  The first tickets scan the
//            occupancy flags for free slots (ascending), the rest look up their
//            chunk of U in slot_of.  Each side is a single-pass scan with
//            decoupled look-back; a union block then takes, for its k-th missing
//            record overall, the k-th free slot from the free-slot blocks'
//            published list, stages the record there and writes the packed
//            copy of every union entry it owns.
// Every status word and free-list entry carries the tag of the call that wrote
// it, so nothing has to be cleared between calls; the last block to finish
// advances the tag and rewinds the two counters.  Union blocks only wait on
// free-slot blocks, which hold earlier tickets and so are already running: no
// wait can depend on a block that has not been dispatched.  Every wait is
// bounded (an error flag is raised instead of hanging).
// Address lists (indirect and sorted modes) are one more coalesced pass over
// the static union ranks of the list entries, plus a per-task sort.
#include <climits>

#include "reorg_dev.h"

namespace gc {
namespace {

using dev::block_excl_scan;
using dev::iload;
using dev::istore;
using dev::kFBlock;
using dev::kLookBack;
using dev::kRThreads;
using dev::kTag;
using dev::kTicket;
using dev::kUBlock;

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Pool reset: slot_of[0, n_ids) = -1 and occ[0, cap) = 0 in one grid.
__global__ void k_pool_reset(int32_t* __restrict__ slot_of, int32_t n_ids, uint32_t* __restrict__ occ, int32_t cap) {
  const int64_t n = n_ids > cap ? n_ids : cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n_ids) slot_of[i] = -1;
    if (i < cap) occ[i] = 0u;
  }
}

__global__ void __launch_bounds__(kRThreads) k_reorg(ReorgArgs a) {
  __shared__ int sh[kRThreads / 64];
  __shared__ int s_ticket;
  __shared__ uint32_t s_tag, s_ex;
  if (threadIdx.x == 0) {
    s_ticket = atomicAdd(a.state + kTicket, 1);
    s_tag = (uint32_t)iload(a.state + kTag) + 1u;
  }
  __syncthreads();
  const int t = s_ticket;
  const uint32_t tag = s_tag;
  if (t < a.nbf)
    dev::free_role<false>(a, t, tag, tag, sh, &s_ex);
  else
  {
    int32_t id[dev::kUItems];
    dev::union_ids(a, t - a.nbf, id);
    dev::union_role<false>(a, t - a.nbf, tag, sh, &s_ex, id);
  }
  // The block with the last ticket rewinds the ticket counter and makes this call's tag the current
  // one: every block has taken its ticket, and has read the tag, since its look-back has seen a tagged
  // word of every earlier union block, and (with free-slot blocks in the launch) the free count, which
  // the last free-slot block writes after seeing one of every earlier free-slot block.
  if (threadIdx.x == 0 && t == a.nbf + a.nbu - 1) {
    if (a.nbf > 0) {
      uint32_t spins = 0;
      while ((uint32_t)(dev::tload(a.ftotal) >> 32) != tag) {
        if (++spins > dev::kSpinLimit) {
          istore(a.state + GC_STATE_ERR, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    istore(a.state + kTicket, 0);
    istore(a.state + kTag, (int32_t)tag);
  }
}

// The wide free-slot scan of a large pool, launched ahead of k_reorg (which then has no free-slot
// blocks): blocks take tickets from their own counter; its look-back words follow the union blocks'.
__global__ void __launch_bounds__(kRThreads) k_free_wide(ReorgArgs a, int32_t nb) {
  __shared__ int sh[kRThreads / 64];
  __shared__ int s_ticket;
  __shared__ uint32_t s_tag, s_ex;
  if (threadIdx.x == 0) {
    s_ticket = atomicAdd(a.state + dev::kWTicket, 1);
    s_tag = (uint32_t)iload(a.state + kTag) + 1u;
  }
  __syncthreads();
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack) + a.nbu;
  dev::free_role_wide(a, flags, s_ticket, nb, s_tag, sh, &s_ex);
  // the block with the last ticket has seen a look-back word of every other block: all have taken
  // their tickets
  if (threadIdx.x == 0 && s_ticket == nb - 1) istore(a.state + dev::kWTicket, 0);
}

// Redundant transfers: every union record is gathered from the source, the pool is not used.
__global__ void k_gather_src(const int32_t* __restrict__ U, int32_t u, const float4* __restrict__ src,
                             float4* __restrict__ packed, int32_t* __restrict__ state) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    state[GC_STATE_UNION] = u;
    state[GC_STATE_MISSING] = u;
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < u; k += gridDim.x * blockDim.x) packed[k] = src[U[k]];
}

// Address lists from the static union ranks of their entries: slot of each entry (0 for an entry
// left without a slot by a full pool; the reorganisation reports that case).
__global__ void k_lists(const int32_t* __restrict__ irank, int64_t n_i, const int32_t* __restrict__ jrank, int64_t n_j,
                        const int32_t* __restrict__ uslot, int32_t* __restrict__ ilist, int32_t* __restrict__ jlist) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_i + n_j; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n_i) {
      const int32_t v = uslot[irank[e]];
      ilist[e] = v > 0 ? v : 0;
    } else {
      const int32_t v = uslot[jrank[e - n_i]];
      jlist[e - n_i] = v > 0 ? v : 0;
    }
  }
}

// Capacity check without side effects: out[0] += missing records of U, out[1] += free slots.
__global__ void __launch_bounds__(256) k_count(const int32_t* __restrict__ U, int32_t u,
                                               const int32_t* __restrict__ slot_of, const uint32_t* __restrict__ occ,
                                               int32_t cap, int32_t* __restrict__ out) {
  __shared__ int sh[4];
  int m = 0, f = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (u > cap ? u : cap);
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k < u && slot_of[U[k]] < 0) ++m;
    if (k < cap && occ[k] == 0u) ++f;
  }
  int tm, tf;
  (void)block_excl_scan(m, sh, &tm);
  (void)block_excl_scan(f, sh, &tf);
  if (threadIdx.x == 0) {
    if (tm) atomicAdd(out, tm);
    if (tf) atomicAdd(out + 1, tf);
  }
}

// Eviction: ids[0, n) leave the pool (n = min(*n_dev, n_host) when n_dev is given).  Ids outside
// [0, n_ids) and ids not resident are skipped.
__global__ void k_evict(const int32_t* __restrict__ ids, const int32_t* __restrict__ n_dev, int32_t n_host,
                        int32_t* __restrict__ slot_of, int32_t n_ids, uint32_t* __restrict__ occ) {
  const int32_t n = n_dev ? min(*n_dev, n_host) : n_host;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t id = ids[k];
    if (id < 0 || id >= n_ids) continue;
    const int32_t s = slot_of[id];
    if (s < 0) continue;
    slot_of[id] = -1;
    occ[s] = 0u;
  }
}

__global__ void k_place(const int32_t* __restrict__ ids, const int32_t* __restrict__ slots, int32_t n,
                        const float4* __restrict__ src, int32_t by_k, float4* __restrict__ pool,
                        int32_t* __restrict__ slot_of, uint32_t* __restrict__ occ) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    int id = ids[k], s = slots[k];
    pool[s] = src[by_k ? k : id];
    slot_of[id] = s;
    occ[s] = 1u;
  }
}

// One block per task: ascending sort of the task's slot list in LDS (bitonic network).
__global__ void __launch_bounds__(256) k_sort_lists(int32_t n_tasks, const int32_t* __restrict__ joff,
                                                    int32_t* __restrict__ jlist) {
  __shared__ int32_t buf[kSortMax];
  for (int t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const int b = joff[t], n = joff[t + 1] - b;
    if (n <= 1) continue;
    int P = 1;
    while (P < n) P <<= 1;
    for (int k = threadIdx.x; k < P; k += blockDim.x) buf[k] = k < n ? jlist[b + k] : INT_MAX;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int k = threadIdx.x; k < P / 2; k += blockDim.x) {
          int lo = 2 * k - (k & (stride - 1));
          int hi = lo + stride;
          bool up = (lo & size) == 0;
          int x = buf[lo], y = buf[hi];
          if ((x > y) == up) {
            buf[lo] = y;
            buf[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) jlist[b + k] = buf[k];
    __syncthreads();
  }
}

inline int grid_for(int64_t n, int per_block, int cap = 65536) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

int union_blocks(int32_t u) { return u > 0 ? (int)(((int64_t)u + kUBlock - 1) / kUBlock) : 1; }

int64_t union_padded(int32_t u) { return (int64_t)union_blocks(u) * kUBlock; }

int free_blocks(int32_t cap) {
  int64_t b = ((int64_t)cap + kFBlock - 1) / kFBlock;
  return b > 0 ? (int)b : 1;
}

// Pools of at least this many narrow free-scan blocks are scanned by the wide form (k_free_wide) in a
// launch of its own: a quarter of the blocks, each at the occupancy of a kernel without union code.
constexpr int kWideFreeBlocks = 512;

static int free_blocks_wide(int32_t cap) {
  int64_t b = ((int64_t)cap + dev::kFWBlock - 1) / dev::kFWBlock;
  return b > 0 ? (int)b : 1;
}

int64_t occ_words(int32_t cap) {
  // one int per slot, padded so that every free-scan thread's load (16 slots, or 64 in the wide form)
  // stays inside the allocation
  return (int64_t)free_blocks_wide(cap) * dev::kFWBlock;
}

int32_t reorg_state_ints(int32_t u, int32_t cap) { return kLookBack + 2 * (union_blocks(u) + free_blocks(cap)); }

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_pool_reset(int32_t* slot_of, int32_t n_ids, uint32_t* occ, int32_t cap, hipStream_t s) {
  int64_t n = n_ids > cap ? n_ids : cap;
  hipLaunchKernelGGL(k_pool_reset, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, slot_of, n_ids, occ, cap);
  return hipGetLastError();
}

hipError_t launch_reorg(ReorgArgs a, hipStream_t s) {
  a.nbu = union_blocks(a.u);
  a.nbf = free_blocks(a.cap);
  a.ftotal = reinterpret_cast<uint64_t*>(a.state + dev::kFreeTotal);
  a.flimit = a.u;
  if (a.nbf >= kWideFreeBlocks) {
    // large pool: the free-slot list first, in its own launch; k_reorg then runs union blocks only
    const int32_t nbw = free_blocks_wide(a.cap);
    hipLaunchKernelGGL(k_free_wide, dim3(nbw), dim3(kRThreads), 0, s, a, nbw);
    a.nbf = 0;
    a.list_ready = 1;
  }
  hipLaunchKernelGGL(k_reorg, dim3(a.nbu + a.nbf), dim3(kRThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_src(const int32_t* U, int32_t u, const float4* src, float4* packed, int32_t* state,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gather_src, dim3(grid_for(u, 256, 4096)), dim3(256), 0, s, U, u, src, packed, state);
  return hipGetLastError();
}

hipError_t launch_lists(const int32_t* irank, int64_t n_i, const int32_t* jrank, int64_t n_j, const int32_t* uslot,
                        int32_t* ilist, int32_t* jlist, hipStream_t s) {
  if (n_i + n_j <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lists, dim3(grid_for(n_i + n_j, 256, 16384)), dim3(256), 0, s, irank, n_i, jrank, n_j, uslot,
                     ilist, jlist);
  return hipGetLastError();
}

hipError_t launch_count(const int32_t* U, int32_t u, const int32_t* slot_of, const uint32_t* occ, int32_t cap,
                        int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(grid_for(u > cap ? u : cap, 256, 2048)), dim3(256), 0, s, U, u, slot_of, occ, cap,
                     out);
  return hipGetLastError();
}

hipError_t launch_evict(const int32_t* ids, const int32_t* n_dev, int32_t n_bound, int32_t* slot_of, int32_t n_ids,
                        uint32_t* occ, hipStream_t s) {
  if (n_bound <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_evict, dim3(grid_for(n_bound, 256, 4096)), dim3(256), 0, s, ids, n_dev, n_bound, slot_of, n_ids,
                     occ);
  return hipGetLastError();
}

hipError_t launch_sort_lists(int32_t n_tasks, const int32_t* joff, int32_t* jlist, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_lists, dim3(grid_for(n_tasks, 1, 8192)), dim3(256), 0, s, n_tasks, joff, jlist);
  return hipGetLastError();
}

hipError_t launch_place(const int32_t* ids, const int32_t* slots, int32_t n, const float4* src, bool by_k, float4* pool,
                        int32_t* slot_of, uint32_t* occ, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_place, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ids, slots, n, src, by_k ? 1 : 0, pool,
                     slot_of, occ);
  return hipGetLastError();
}

}  // namespace gc
