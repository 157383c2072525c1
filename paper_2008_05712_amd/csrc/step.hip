// Whole-step persistent kernel (the batched form): one launch runs every round
// of a step -- the round's reorganisation (free-slot scan, chare-table lookup,
// slot assignment, staging, packing, and with the evicting fixture the
// eviction of what it staged; Sec. 3.2) and its combined force pass
// (Sec. 3.1) -- so the rounds need no kernel boundaries and the passes of
// consecutive rounds overlap.  (The eviction of what the previous step's last
// round left staged runs as a small kernel before the launch.)
//
// Work items are numbered in ticket order:
//   free(0) union(0) union(1) union(2) union(3) force(0) union(4) force(1) ...
//   union(R-1) force(R-4) force(R-3) force(R-2) force(R-1)
// so the reorganisation chain runs kStepLead = 3 rounds ahead of the force
// passes (the chain is sequential -- each round's lookup sees the pool as the
// round before left it -- and latency-bound, the passes are throughput-bound;
// measured: a lead of 1 round is 14 % slower than 2, and 3 is 2 % faster
// than 2, as fast as 4).
//
// The free-slot list is scanned once, in round 0.  Inside the launch only the
// union items change the occupancy: a round takes the lowest free slots in
// order, so the free slots at the start of round r are round 0's list without
// the entries taken (and kept) by earlier rounds -- an offset into that list,
// which is 0 throughout when each round evicts what it stages.
//
// A union item has a table part (lookup, missing ranks, slot assignment, the
// chare-table and occupancy updates), which is all the next round's lookup
// depends on, and a data part (record loads, packed copies, staging of the
// records into their slots), counted separately.  A block takes tickets from a
// device counter (the next one is requested while the current item runs) and
// waits only for items with smaller tickets:
//   free(0) union(r)  table parts wait for the table parts of the previous
//                     round with chain items; inside round 0 on the free-slot
//                     list and look-back words as in the per-batch kernel;
//   union(r) data     waits for the previous round's data parts (pool records
//                     it stages may be read or its slots reused);
//   force(r)          waits for the data parts of round r.
// With the evicting fixture a round changes no value of the chare table, the occupancy or the resident
// records (a staged id's entry and its slot's flag are rewritten with what they held, and the records
// go into free slots that no lookup reaches), so every round sees the pool as the launch found it:
// rounds after the first wait for nothing but round 0's free-slot count, probe its list entries as
// they appear, and read the table and records with plain loads.
// The unfinished item with the smallest ticket therefore always progresses (its
// dependencies are finished), so the grid never deadlocks whatever the order
// in which its blocks run; every wait is bounded anyway and raises an error
// flag.  Counters are monotonic across launches (a launch epoch scales the
// targets), so nothing is cleared between replays; the last block out
// advances the epoch.  Reorganisation items raise their waves' issue priority
// while they run: they are latency-bound and on the step's critical path.
//
// Memory: the chare table, occupancy flags, resident pool records and missing
// lists are read with device-scope coherent (sc1) loads (the L2 of one XCD is
// not coherent with the others'); every item writes plainly and, before it is
// counted done, writes its XCD's L2 back (device-scope release).  Items of one
// round exchange only tagged words, through device-scope atomics.  A force
// item reads a round's packed records only after that round's data parts are
// all done; no earlier access in the launch touches those lines (each union
// item writes whole lines of its own), so its caches hold no stale copy.
#include "grav_dev.h"
#include "reorg_dev.h"

namespace gc {
namespace {

using dev::grav_lds_per_wave;
using dev::uniform;

// The thread that requests tickets and loads the next item: the first lane of the last wavefront,
// which issues no global stores in a force item, so its end-of-item wait for the ticket and the
// item covers nothing else (wavefront 0 writes the accelerations).
constexpr int kOwner = dev::kRThreads - 64;

__device__ __forceinline__ void wait_ge(uint64_t* p, uint64_t target, int32_t* err, uint32_t limit) {
  uint32_t spins = 0;
  while (dev::tload(p) < target) {
    if (++spins > limit) {
      dev::istore(err, 1);
      return;
    }
    // back off: many blocks may wait on one counter, and its line is also the one being counted up
    if (spins < 4)
      __builtin_amdgcn_s_sleep(2);
    else
      __builtin_amdgcn_s_sleep(16);
  }
}

// Counts the item done.  With `release` every wave first waits for its own stores to reach the L2,
// then one thread writes the L2 back (device-scope release), so that an item that waits for the count
// reads what this one wrote.  Without it only the count is published (nothing in the launch reads the
// item's plain stores; tagged words are device-scope atomics and need no release).
__device__ __forceinline__ uint64_t publish_done(uint64_t* ctr, bool release) {
  if (release) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  uint64_t old = 0;
  if (threadIdx.x == 0) {
    if (release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    old = atomicAdd(reinterpret_cast<unsigned long long*>(ctr), 1ull);
  }
  return old;
}

// Values read from LDS by every lane, marked wavefront-uniform so that they live in scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The per-round arguments are never written during the launch: read through the constant address
// space, with a uniform round index they come in by scalar loads (scalar cache) into scalar registers.
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

// FORCE: the launch runs force items (5 waves per SIMD: at most 96 VGPRs for the force code);
// without (the rounds schedule's reorganisation launch) no force code is compiled in and the
// reorganisation items get the registers they use.
template <int ORDER, int TPL, bool FORCE>
__global__ void __launch_bounds__(dev::kRThreads) __attribute__((amdgpu_waves_per_eu(FORCE ? 5 : 1))) k_step(StepArgs s) {
  extern __shared__ float4 smem[];
  __shared__ int sh[dev::kRThreads / 64];
  __shared__ uint32_t s_ex, s_tag;
  __shared__ int64_t s_base, s_avail;
  __shared__ int64_t s_tk, s_tn;                 // the block's current ticket and the next (this launch's)
  __shared__ __align__(16) StepItem s_item[2];   // its item and the next one, alternately
  __shared__ uint64_t s_epoch;
  const int tid = threadIdx.x;
  if (tid == 0) s_epoch = dev::tload(s.ctr + kCtrStride * kCtrEpoch);
  __syncthreads();
  const uint64_t E = s_epoch;
  // every block takes tickets until it holds one past the last item
  const uint64_t base = E * ((uint64_t)s.n_items + gridDim.x);  // tickets taken by earlier launches
  const uint64_t goal = E + 1;
  const uint32_t ltag = (uint32_t)goal;  // tag of this launch's free-slot list words
  unsigned long long* tickets = reinterpret_cast<unsigned long long*>(s.ctr + kCtrStride * kCtrTickets);
  if (tid == 0) {
    const int64_t t0 = (int64_t)(atomicAdd(tickets, 1ull) - base);
    s_tk = t0;
    if (t0 < s.n_items) s_item[0] = s.items[t0];
  }
  __syncthreads();
  int cb = 0;
  int ready = -1;  // this block has seen the data parts of rounds <= ready complete
  // a force item followed by a force item loads the next one's first node tile and (thread 0) its
  // round's data-part count while it finishes
  dev::NodePrefetch<ORDER> pf;
  bool have_pf = false;
  int poll_k = -1;
  uint64_t poll_v = 0;
  while (true) {
    const int64_t t = s_tk;
    if (t >= s.n_items) break;
    const int kind = uni(s_item[cb].kind);
    const int type = kind & 3;
    const int k = kind >> 2;
    const int idx = uni(s_item[cb].idx);
    // the next ticket is requested now and its item loaded straight into the other LDS slot once
    // the ticket is back (fetch_next, called by every thread: inside a force item once its first
    // loads are out, else at the end); neither is waited for before the end of this item
    unsigned long long nxt = 0;
    if (tid == kOwner) nxt = atomicAdd(tickets, 1ull);
    auto fetch_next = [&] {
      if ((tid >> 6) == (kOwner >> 6)) {
        const uint64_t v = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(nxt >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)nxt);
        const int64_t tn = (int64_t)(v - base);
        if ((unsigned)(tid - kOwner) < 2u && tn < s.n_items)
          __builtin_amdgcn_global_load_lds(reinterpret_cast<const char*>(s.items + tn) + 16 * (tid - kOwner),
                                           (void __attribute__((address_space(3)))*)&s_item[cb ^ 1], 16, 0, 0);
      }
    };
    const __attribute__((address_space(4))) StepRound& R = cst(s.rounds)[k];
    int32_t* err = R.reorg.state + GC_STATE_ERR;
    uint64_t* ch_done = s.ctr + kCtrStride * (kCtrRounds + 2 * k);
    uint64_t* dt_done = ch_done + kCtrStride;
    const int pr = uniform(R.prev);
    if (FORCE && type == kItemForce) {
      const GravArgs ga = cload(&R.grav);
      const dev::TaskDesc td{uni(s_item[cb].i_begin), uni(s_item[cb].i_count), uni(s_item[cb].j_first),
                             uni(s_item[cb].j_nranges), uni(s_item[cb].n_first), uni(s_item[cb].n_count), idx};
      // (the test hook's round waits for one data part more than exist, so its waits give up)
      const uint64_t target = goal * (uint64_t)R.reorg.nbu + (k == s.fail_round ? 1u : 0u);
      bool pf_next = false;
      // the round's packed records are read only once its data parts are done
      dev::grav_task<ORDER, false, TPL>(ga, 0, td, smem, pf, have_pf, [&] {
        if (k > ready) {
          if (tid == 0 && !(poll_k == k && poll_v >= target))
            wait_ge(dt_done, target, err, k == s.fail_round ? s.fail_spins : s.spin_limit);
          __syncthreads();
          ready = k;
        }
        fetch_next();
      }, [&](int phase) {
        if (phase == 0) {
          if (tid == kOwner) {
            __builtin_amdgcn_s_waitcnt(0);  // the next item has landed in LDS
            s_tn = (int64_t)(nxt - base);
          }
          return;
        }
        const int64_t t2 = s_tn;
        if (t2 >= s.n_items) return;
        const int kind2 = uni(s_item[cb ^ 1].kind);
        if ((kind2 & 3) != kItemForce) return;
        const int k2 = kind2 >> 2;
        const __attribute__((address_space(4))) StepRound& R2 = cst(s.rounds)[k2];
        dev::node_prefetch<ORDER>(dev::node_rsrc(R2.grav.nodes, R2.grav.n_nodes), R2.grav.node_idx, uni(s_item[cb ^ 1].n_first),
                                  uni(s_item[cb ^ 1].n_count), pf);
        pf_next = true;
        if (tid == 0 && k2 > ready) {
          poll_k = k2;
          poll_v = dev::tload(s.ctr + kCtrStride * (kCtrRounds + 2 * k2 + 1));
        }
      });
      have_pf = pf_next;
    } else {
      // reorganisation items are on the critical path of the step and latency-bound: their waves
      // issue ahead of the force waves sharing the CU
      __builtin_amdgcn_s_setprio(3);
      const ReorgArgs ra = cload(&R.reorg);
      int32_t ids[dev::kUItems];
      if (type == kItemUnion) dev::union_ids(ra, idx, ids);  // static: loaded while the dependencies finish
      if (tid == 0) {
        int64_t fbase = 0, favail = -1;
        if (pr >= 0) {
          wait_ge(s.ctr + kCtrStride * (kCtrRounds + 2 * pr), goal * (uint64_t)cst(s.rounds)[pr].n_chain, err,
                  s.spin_limit);
          // round 0 is complete: the launch's free count is known; this round's offset into the list is
          // the previous one plus what that round took and kept
          const uint64_t ft = dev::tload(s.fmeta);
          if ((uint32_t)(ft >> 32) != ltag) dev::istore(err, 1);
          const int64_t F = (int64_t)(ft & 0x7fffffffu);
          if (!ra.evict_after && cst(s.rounds)[pr].reorg.nbu > 0) {
            const uint64_t bw = dev::tload(s.fmeta + 1 + pr);
            if ((uint32_t)(bw >> 32) != ltag) dev::istore(err, 1);
            const int64_t bp = (int64_t)(bw & 0x7fffffffu);
            const int64_t mp = dev::iload(cst(s.rounds)[pr].reorg.state + GC_STATE_MISSING);
            const int64_t avail = F - bp > 0 ? F - bp : 0;
            fbase = bp + (mp < avail ? mp : avail);
          }
          favail = F - fbase;
        }
        // an independent round (pr == kPrevFreeList) waits for nothing here: its list entries are
        // probed as they appear, and its last union item records the launch's free count at its end
        s_base = fbase;
        s_avail = favail;
        s_tag = (uint32_t)dev::iload(R.reorg.state + dev::kTag) + 1u;
      }
      __syncthreads();
      const uint32_t tag = s_tag;
      if (type == kItemFree) {
        // plain loads: no item of the launch writes the occupancy of a slot before its free-scan item
        // has listed it (slots are taken from the list), and the launch starts after every earlier write
        dev::free_role<false>(ra, idx, tag, ltag, sh, &s_ex);
        // without the fixture later rounds wait for this count, then read the list's count (a tagged
        // word; the release orders it before the count), else they poll that word itself
        const uint64_t old = publish_done(ch_done, !ra.evict_after);
        if (tid == 0 && old + 1 == goal * (uint64_t)R.n_chain) dev::istore(R.reorg.state + dev::kTag, (int32_t)tag);
      } else {
        int32_t slot[dev::kUItems];
        uint32_t fm = 0;
        const int64_t fbase = s_base;
        // with the fixture and no force items in the launch, both parts in one pass (in a kernel with
        // force code its registers would spill); otherwise the table part first
        const bool fused = !FORCE && ra.evict_after;
        if (fused) dev::union_fused(ra, idx, tag, ltag, fbase, sh, &s_ex, ids);
        else (void)dev::union_table(ra, idx, tag, ltag, fbase, sh, &s_ex, ids, slot, fm, !ra.evict_after);
        if (tid == 0 && idx == ra.nbu - 1) {
          dev::tstore(s.fmeta + 1 + k, dev::tword(ltag, 0, (uint32_t)fbase));
          if (s_avail >= 0) dev::istore(R.reorg.state + GC_STATE_FREE, (int32_t)s_avail);
          if (pr == kPrevFreeList) {
            // the launch's free count, which round 0's last free-scan item writes (tagged); the probes
            // above have found their entries, so it is written or about to be
            uint64_t ft = dev::tload(s.fmeta);
            for (uint32_t spins = 0; (uint32_t)(ft >> 32) != ltag; ft = dev::tload(s.fmeta)) {
              if (++spins > s.spin_limit) {
                dev::istore(err, 1);
                break;
              }
              __builtin_amdgcn_s_sleep(2);
            }
            dev::istore(R.reorg.state + GC_STATE_FREE, (int32_t)(ft & 0x7fffffffu));
          }
        }
        if (fused) {
          // both parts are done; nothing in the launch reads the records, and the table part's count
          // only advances the batch's tag
          (void)publish_done(dt_done, false);
          const uint64_t old = publish_done(ch_done, false);
          if (tid == 0 && old + 1 == goal * (uint64_t)R.n_chain) dev::istore(R.reorg.state + dev::kTag, (int32_t)tag);
        } else {
          // later rounds read this round's table writes unless the fixture leaves the table unchanged
          const uint64_t old = publish_done(ch_done, !ra.evict_after);
          if (tid == 0 && old + 1 == goal * (uint64_t)R.n_chain) dev::istore(R.reorg.state + dev::kTag, (int32_t)tag);
          // data part: after the previous round's (its staging may be read here, its slots reused)
          if (tid == 0 && pr >= 0)
            wait_ge(s.ctr + kCtrStride * (kCtrRounds + 2 * pr + 1), goal * (uint64_t)cst(s.rounds)[pr].reorg.nbu, err,
                    s.spin_limit);
          __syncthreads();
          dev::union_data(ra, idx, ids, slot, fm, !ra.evict_after);
          // read by this round's force items, and without the fixture by later rounds' data parts
          (void)publish_done(dt_done, s.has_force || !ra.evict_after);
        }
      }
      __builtin_amdgcn_s_setprio(0);
      fetch_next();
    }
    if (tid == kOwner) {
      __builtin_amdgcn_s_waitcnt(0);  // the next item has landed in LDS
      s_tk = (int64_t)(nxt - base);
    }
    __syncthreads();
    cb ^= 1;
  }
  if (tid == 0 && atomicAdd(reinterpret_cast<unsigned long long*>(s.ctr + kCtrStride * kCtrExits), 1ull) + 1 ==
                      goal * gridDim.x)
    dev::tstore(s.ctr + kCtrStride * kCtrEpoch, goal);
}

size_t step_lds(int tile) { return (size_t)(dev::kRThreads / 64) * grav_lds_per_wave(tile) * sizeof(float4); }

template <int ORDER, int TPL>
hipError_t step_attr(int tile) {
  const size_t lds = step_lds(tile);
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_step<ORDER, TPL, true>), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <int ORDER, int TPL>
hipError_t step_launch_one(const StepArgs& a, int grid, int tile, hipStream_t s) {
  hipError_t e = step_attr<ORDER, TPL>(tile);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_step<ORDER, TPL, true>), dim3(grid), dim3(dev::kRThreads), step_lds(tile), s, a);
  return hipGetLastError();
}

template <int ORDER, int TPL>
hipError_t step_occ_one(int tile, int* blocks) {
  hipError_t e = step_attr<ORDER, TPL>(tile);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_step<ORDER, TPL, true>, dev::kRThreads, step_lds(tile));
}

}  // namespace

hipError_t launch_step_reorg(const StepArgs& a, int grid, hipStream_t s) {
  if (grid < 1 || a.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_step<2, 1, false>), dim3(grid), dim3(dev::kRThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_step(int order, int tpl, const StepArgs& a, int grid, int tile, hipStream_t s) {
  if (grid < 1 || a.n_items <= 0) return hipSuccess;
  if (order == 1) {
    if (tpl == 2) return step_launch_one<1, 2>(a, grid, tile, s);
    if (tpl == 3) return step_launch_one<1, 3>(a, grid, tile, s);
    return step_launch_one<1, 1>(a, grid, tile, s);
  }
  if (tpl == 2) return step_launch_one<2, 2>(a, grid, tile, s);
  if (tpl == 3) return step_launch_one<2, 3>(a, grid, tile, s);
  return step_launch_one<2, 1>(a, grid, tile, s);
}

hipError_t step_occupancy(int order, int tpl, int tile, int* blocks) {
  if (order == 1) {
    if (tpl == 2) return step_occ_one<1, 2>(tile, blocks);
    if (tpl == 3) return step_occ_one<1, 3>(tile, blocks);
    return step_occ_one<1, 1>(tile, blocks);
  }
  if (tpl == 2) return step_occ_one<2, 2>(tile, blocks);
  if (tpl == 3) return step_occ_one<2, 3>(tile, blocks);
  return step_occ_one<2, 1>(tile, blocks);
}

}  // namespace gc
