// Device code of the reorganisation (Sec. 3.2), shared by the per-batch
// kernels and the whole-step persistent kernel: the tagged single-pass scans
// and the free-slot and union (lookup, slot assignment, staging, packing)
// roles of a block.
//
// Inside the whole-step kernel (COH = true) other blocks change the chare
// table, the occupancy flags and the pool between rounds, and the L2 of one XCD
// is not coherent with the others': there the roles read those with
// device-scope coherent (sc1) loads, and the kernel writes its L2 back (a
// device-scope release) before it counts an item done.  The per-batch kernel
// (COH = false) never reads in-kernel what another block wrote to them and uses
// plain loads.  Items of one round exchange only tagged words (look-back,
// free-slot list, totals), through device-scope atomics.
#pragma once

#include "gc_internal.h"
#include "mem_dev.h"

namespace gc {
namespace dev {

constexpr int kRThreads = 256;                      // threads of every reorganisation block
#ifndef GC_UITEMS
#define GC_UITEMS 8
#endif
constexpr int kUItems = GC_UITEMS;                  // union entries per thread (a multiple of 4)
constexpr int kUBlock = kRThreads * kUItems;        // union entries per block
constexpr int kFItems = 16;                         // occupancy entries per thread
constexpr int kFBlock = kRThreads * kFItems;        // pool slots per free-scan block
constexpr int kFWItems = 64;                        // occupancy entries per thread, wide free scan
constexpr int kFWBlock = kRThreads * kFWItems;      // pool slots per wide free-scan block
constexpr uint32_t kSpinLimit = 1u << 22;           // bound on every wait: each wave exits

// state[] layout (int32 units): the host-visible words (gc_internal.h), the call tag and the free
// count on the first 128-byte line; each ticket counter on a line of its own (every block of a call
// adds to its counter, and atomics on one line are serialised where they are performed); the
// look-back words from the fourth line on.
constexpr int kTag = 10, kFreeTotal = 12, kTicket = 32, kWTicket = 64, kLookBack = 96;

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across the block; block total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int* sh_wave, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) sh_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    int s = sh_wave[k];
    off += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Tagged 64-bit words: bits 0-30 a count, bit 31 a flag, bits 32-63 the call tag.  Relaxed
// device-scope atomics: each word carries its own payload, nothing else is published through it
// (acquire/release here would write back and invalidate the caches on every probe).
__device__ __forceinline__ uint64_t tword(uint32_t tag, uint32_t flag, uint32_t cnt) {
  return ((uint64_t)tag << 32) | ((uint64_t)flag << 31) | (uint64_t)cnt;
}
__device__ __forceinline__ void tstore(uint64_t* p, uint64_t v) { astore(p, v); }
__device__ __forceinline__ uint64_t tload(uint64_t* p) { return aload(p); }
__device__ __forceinline__ int32_t iload(int32_t* p) { return aload(p); }
__device__ __forceinline__ void istore(int32_t* p, int32_t v) { astore(p, v); }

// Wavefront 0 of chain block `bid`: publish the block aggregate, look back over up to 64
// predecessors per probe (a word of another call counts as not yet written; the run up to the
// nearest inclusive prefix is summed once all of it is written), publish the inclusive prefix,
// return the exclusive prefix.
__device__ __forceinline__ uint32_t look_back(uint64_t* flags, int bid, uint32_t tag, uint32_t agg, int32_t* err) {
  const int lane = threadIdx.x & 63;
  if (bid == 0) {
    if (lane == 0) tstore(flags, tword(tag, 1, agg));
    return 0;
  }
  if (lane == 0) tstore(flags + bid, tword(tag, 0, agg));
  uint32_t x = 0, spins = 0;
  int hi = bid - 1;
  while (true) {
    const int j = hi - lane;
    const uint64_t w = j >= 0 ? tload(flags + j) : tword(tag, 1, 0);  // before block 0: a zero prefix
    const bool mine = (uint32_t)(w >> 32) == tag;
    const uint64_t pre = __ballot(mine && ((w >> 31) & 1u));
    const uint64_t emp = __ballot(!mine);
    const int stop = pre ? __builtin_ctzll(pre) : 63;  // last lane of the run to sum
    const uint64_t run = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
    if (emp & run) {
      if (++spins > kSpinLimit) {
        if (lane == 0) istore(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint32_t v = lane <= stop ? (uint32_t)(w & 0x7fffffffu) : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    x += v;
    if (pre) break;
    hi -= 64;
  }
  if (lane == 0) tstore(flags + bid, tword(tag, 1, x + agg));
  return x;
}

template <bool COH>
__device__ __forceinline__ int32_t ld_i32(const int32_t* p) {
  if (COH) return iload(const_cast<int32_t*>(p));
  return gld(p);
}

// One 16-byte record; COH: two device-scope 8-byte loads.
template <bool COH>
__device__ __forceinline__ float4 ld_rec(const float4* p) {
  if (!COH) return gld(p);
  uint64_t* q = reinterpret_cast<uint64_t*>(const_cast<float4*>(p));
  const uint64_t lo = tload(q), hi = tload(q + 1);
  return make_float4(__uint_as_float((uint32_t)lo), __uint_as_float((uint32_t)(lo >> 32)),
                     __uint_as_float((uint32_t)hi), __uint_as_float((uint32_t)(hi >> 32)));
}

// Free-slot side: the lowest free slots in ascending order, listed up to a.flimit entries (at least
// the number of records that can go missing); the last block publishes the pool's free count.
// Look-back words carry `tag`, list entries and the free count `ltag`.
template <bool COH>
__device__ __forceinline__ void free_role(const ReorgArgs& a, int b, uint32_t tag, uint32_t ltag, int* sh,
                                          uint32_t* s_ex) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack);
  const int64_t s0 = (int64_t)b * kFBlock + (int64_t)threadIdx.x * kFItems;
  uint32_t f = 0;
  if (s0 < a.cap) {
    if (COH) {
      const int32_t* o = reinterpret_cast<const int32_t*>(a.occ) + s0;
#pragma unroll
      for (int k = 0; k < kFItems; ++k)
        if (ld_i32<true>(o + k) == 0 && s0 + k < a.cap) f |= 1u << k;
    } else {
      const int4* o4 = reinterpret_cast<const int4*>(a.occ + s0);  // occ is padded to whole blocks
#pragma unroll
      for (int q = 0; q < kFItems / 4; ++q) {
        const int4 o = gld(o4 + q);
        const uint32_t ov[4] = {(uint32_t)o.x, (uint32_t)o.y, (uint32_t)o.z, (uint32_t)o.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (ov[k] == 0u && s0 + 4 * q + k < a.cap) f |= 1u << (4 * q + k);
      }
    }
  }
  int tot;
  int r = block_excl_scan(__popc(f), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbf - 1) {
        tstore(a.ftotal, tword(ltag, 0, ex + (uint32_t)tot));
        istore(a.state + GC_STATE_FREE, (int32_t)(ex + (uint32_t)tot));
      }
    }
  }
  __syncthreads();
  r += (int)*s_ex;
  if (r >= a.flimit) return;
#pragma unroll
  for (int k = 0; k < kFItems; ++k)
    if ((f >> k) & 1u) {
      if (r < a.flimit) tstore(a.free_list + r, tword(ltag, 0, (uint32_t)(s0 + k)));
      ++r;
    }
}

// Wide form of the free-slot side, for large pools, in a launch of its own ahead of the union side:
// 64 slots a thread, so a quarter of the blocks (each a chain step of the look-back) and no union
// code's registers.  flags: this launch's look-back words (nb of them).  The list and its count are
// the narrow form's tagged words; the list is written with plain stores, as the union side reads it
// only in a later launch (ReorgArgs::list_ready).  (Untagged 4-byte entries bounded by the count
// were measured 10 % slower on the 2^26-slot pool.)
__device__ __forceinline__ void free_role_wide(const ReorgArgs& a, uint64_t* flags, int b, int nb, uint32_t tag,
                                               int* sh, uint32_t* s_ex) {
  const int64_t s0 = (int64_t)b * kFWBlock + (int64_t)threadIdx.x * kFWItems;
  uint64_t f = 0;
  if (s0 < a.cap) {
    const int4* o4 = reinterpret_cast<const int4*>(a.occ + s0);  // occ is padded to whole wide blocks
#pragma unroll
    for (int q = 0; q < kFWItems / 4; ++q) {
      const int4 o = gld(o4 + q);
      const uint32_t ov[4] = {(uint32_t)o.x, (uint32_t)o.y, (uint32_t)o.z, (uint32_t)o.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (ov[k] == 0u && s0 + 4 * q + k < a.cap) f |= 1ull << (4 * q + k);
    }
  }
  int tot;
  int r = block_excl_scan(__popcll(f), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == nb - 1) {
        tstore(a.ftotal, tword(tag, 0, ex + (uint32_t)tot));
        istore(a.state + GC_STATE_FREE, (int32_t)(ex + (uint32_t)tot));
      }
    }
  }
  __syncthreads();
  r += (int)*s_ex;
  // only the first flimit free slots are listed (no request takes more)
  while (f && r < a.flimit) {
    const int k = __builtin_ctzll(f);
    f &= f - 1;
    gst(a.free_list + r, tword(tag, 0, (uint32_t)(s0 + k)));
    ++r;
  }
}

// Union side: residency of this block's chunk of U, the missing ranks, then slot assignment,
// staging and the packed copies.
// This thread's union ids of union block b (U is fixed at commit, so they may be loaded before the
// block's dependencies are complete).
__device__ __forceinline__ void union_ids(const ReorgArgs& a, int b, int32_t (&id)[kUItems]) {
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  const int4* u4 = reinterpret_cast<const int4*>(a.U + k0);  // U is padded to whole blocks
#pragma unroll
  for (int q = 0; q < kUItems / 4; ++q) {
    const int4 x = gld(u4 + q);
    id[4 * q] = x.x; id[4 * q + 1] = x.y; id[4 * q + 2] = x.z; id[4 * q + 3] = x.w;
  }
}

// Chare-table lookup of this thread's entries: resident slot (sl) and the missing mask.
template <bool COH>
__device__ __forceinline__ uint32_t union_lookup(const ReorgArgs& a, int b, const int32_t (&id)[kUItems],
                                                 int32_t (&sl)[kUItems]) {
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  uint32_t fm = 0;
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    sl[i] = 0;
    if (k0 + i < a.u) {
      sl[i] = ld_i32<COH>(a.slot_of + id[i]);
      if (sl[i] < 0) fm |= 1u << i;
    }
  }
  return fm;
}

// Entry j of the free-slot list for the missing entries of mask fm, in order from list index r0
// (entries carry `ltag` once listed; *ftotal, once it carries `ltag`, bounds the list; the list
// holds `lim` entries, and an index at or beyond it is past the pool's free slots): one probe for
// all of them in flight, then a bounded wait that re-probes those still unlisted.  Writes the slot
// (or -1: the pool has no free slot for it) into slot[i] for each missing i.
__device__ __forceinline__ void union_probe(uint64_t* flist, uint64_t* ftotal, uint32_t ltag, int64_t r0, int64_t lim,
                                            uint32_t fm, int32_t (&slot)[kUItems], int32_t* err, bool ready = false) {
  if (ready) {
    // the list is complete: an entry without the tag lies past the pool's free slots
    int64_t r = r0;
#pragma unroll
    for (int i = 0; i < kUItems; ++i)
      if ((fm >> i) & 1u) {
        slot[i] = -1;
        if (r < lim) {
          const uint64_t w = gld(flist + r);
          if ((uint32_t)(w >> 32) == ltag) slot[i] = (int32_t)(w & 0x7fffffffu);
        }
        ++r;
      }
    return;
  }
  uint32_t pend = 0;
  {
    int64_t r = r0;
#pragma unroll
    for (int i = 0; i < kUItems; ++i) {
      if ((fm >> i) & 1u) {
        slot[i] = -1;
        if (r < lim) {
          const uint64_t w = tload(flist + r);
          if ((uint32_t)(w >> 32) == ltag) slot[i] = (int32_t)(w & 0x7fffffffu);
          else pend |= 1u << i;
        }
        ++r;
      }
    }
  }
  uint32_t spins = 0;
  while (pend) {
    if (++spins > kSpinLimit) {
      istore(err, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    const uint64_t t = tload(ftotal);
    const bool total_known = (uint32_t)(t >> 32) == ltag;
    int64_t r = r0;
#pragma unroll
    for (int i = 0; i < kUItems; ++i)
      if ((fm >> i) & 1u) {
        if ((pend >> i) & 1u) {  // (r < lim: only such entries are pending)
          const uint64_t w = tload(flist + r);
          if ((uint32_t)(w >> 32) == ltag) {
            slot[i] = (int32_t)(w & 0x7fffffffu);
            pend &= ~(1u << i);
          } else if (total_known && r >= (int64_t)(t & 0x7fffffffu)) {
            pend &= ~(1u << i);  // the pool has no free slot for this one
          }
        }
        ++r;
      }
  }
}

// Per-batch form of the union side: lookup, then every entry's record -- from the pool if resident,
// from the source if missing -- is loaded before the ranks are known and its packed copy written at
// once (neither waits for the scans); then the missing ranks, slot assignment and staging.  With a
// host-staged batch (a.staged) a missing record sits at its missing rank in a.staged, so it is
// loaded, packed and staged once the rank is known.
template <bool COH>
__device__ __forceinline__ void union_role(const ReorgArgs& a, int b, uint32_t tag, int* sh, uint32_t* s_ex,
                                           const int32_t (&id)[kUItems]) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack) + a.nbf;
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  const bool stg = a.staged != nullptr;
  int32_t sl[kUItems];
  const uint32_t fm = union_lookup<COH>(a, b, id, sl);
  float rx[kUItems], ry[kUItems], rz[kUItems], rw[kUItems];
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((fm >> i) & 1u) {
      if (!stg) v = gld(a.src + id[i]);
    } else if (k0 + i < a.u) {
      v = ld_rec<COH>(a.pool + sl[i]);
    }
    rx[i] = v.x;
    ry[i] = v.y;
    rz[i] = v.z;
    rw[i] = v.w;
  }
  int tot;
  int rm = block_excl_scan(__popc(fm), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbu - 1) {
        istore(a.state + GC_STATE_UNION, a.u);
        istore(a.state + GC_STATE_MISSING, (int32_t)(ex + (uint32_t)tot));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    const int64_t k = k0 + i;
    if (k < a.u) {
      const bool miss = (fm >> i) & 1u;
      if (!miss) gst(a.uslot + k, sl[i]);
      if (a.pack && !(stg && miss)) gst(a.packed + k, make_float4(rx[i], ry[i], rz[i], rw[i]));
    }
  }
  __syncthreads();
  if (!fm) return;
  rm += (int)*s_ex;
  if (stg) {
    int r = rm;
#pragma unroll
    for (int i = 0; i < kUItems; ++i)
      if ((fm >> i) & 1u) {
        const float4 v = gld(a.staged + r);
        rx[i] = v.x;
        ry[i] = v.y;
        rz[i] = v.z;
        rw[i] = v.w;
        if (a.pack) gst(a.packed + k0 + i, v);
        ++r;
      }
  }
  // the rm-th free slot for the rm-th missing record, once its free-scan block has listed it
  union_probe(a.free_list, a.ftotal, tag, rm, a.flimit, fm, sl, a.state + GC_STATE_ERR, a.list_ready != 0);
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    if (!((fm >> i) & 1u)) continue;
    const int64_t k = k0 + i;
    const int32_t s = sl[i];
    gst(a.missing + rm, id[i]);
    gst(a.mslot + rm, s);
    gst(a.uslot + k, s);
    if (s >= 0) {
      gst(a.pool + s, make_float4(rx[i], ry[i], rz[i], rw[i]));
      gst(a.slot_of + id[i], s);
      gst(a.occ + s, 1u);
    }
    ++rm;
  }
}

// Whole-step form of the union side, in two parts.  The table part -- lookup, missing ranks, slot
// assignment and the table updates (and, with evict_after, the eviction of what it stages) -- is all
// the next round's lookup depends on.  The data part -- record loads, packed copies, staging of the
// missing records into their slots -- only feeds this round's pass and later rounds' pool reads, so
// it runs after the table part has been published.  slot[i] leaves the table part as the entry's
// slot (resident: its slot; missing: the assigned slot or -1) and fm as the missing mask.
// Returns the round's missing count on the last union block's thread 0 (0 elsewhere).
// coh: the chare table and resident records are read with device-scope coherent loads, as earlier
// rounds of the launch may have changed them; with evict_after no round changes a value of either
// (a staged id's entry and slot flag are rewritten with what they hold, and staged slots are free
// slots that no lookup reaches), so plain loads read the same values.
__device__ __forceinline__ uint32_t union_table(const ReorgArgs& a, int b, uint32_t tag, uint32_t ltag,
                                                int64_t fbase, int* sh, uint32_t* s_ex, const int32_t (&id)[kUItems],
                                                int32_t (&slot)[kUItems], uint32_t& fm, bool coh) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack) + a.nbf;
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  fm = coh ? union_lookup<true>(a, b, id, slot) : union_lookup<false>(a, b, id, slot);
  int tot;
  int rm = block_excl_scan(__popc(fm), sh, &tot);
  uint32_t m = 0;
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbu - 1) {
        m = ex + (uint32_t)tot;
        istore(a.state + GC_STATE_UNION, a.u);
        istore(a.state + GC_STATE_MISSING, (int32_t)m);
      }
    }
  }
  __syncthreads();
  rm += (int)*s_ex;
  if (fm) union_probe(a.free_list, a.ftotal, ltag, fbase + rm, a.flimit, fm, slot, a.state + GC_STATE_ERR);
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    const int64_t k = k0 + i;
    if (k >= a.u) continue;
    const int32_t s = slot[i];
    gst(a.uslot + k, s);
    if ((fm >> i) & 1u) {
      gst(a.missing + rm, id[i]);
      gst(a.mslot + rm, s);
      ++rm;
      if (s >= 0) {
        // staged, and with evict_after at once evicted again (the pool keeps its base residency
        // between rounds); the record itself is written by the data part
        gst(a.slot_of + id[i], a.evict_after ? -1 : s);
        gst(a.occ + s, a.evict_after ? 0u : 1u);
      }
    }
  }
  return m;
}

// Whole-step form of the union side with evict_after, both parts in one pass: no round of the launch
// changes a value of the chare table, the occupancy or a resident record, so the records are loaded
// right after the lookup, and arrive while the missing ranks and slot assignment are found; then the
// packed copies and the staging.  A staged id's chare-table entry and slot flag end as they
// were, so neither is written.
__device__ __forceinline__ void union_fused(const ReorgArgs& a, int b, uint32_t tag, uint32_t ltag, int64_t fbase,
                                            int* sh, uint32_t* s_ex, const int32_t (&id)[kUItems]) {
  uint64_t* flags = reinterpret_cast<uint64_t*>(a.state + kLookBack) + a.nbf;
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  int32_t slot[kUItems];
  const uint32_t fm = union_lookup<false>(a, b, id, slot);
  float4 v[kUItems];
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((fm >> i) & 1u) v[i] = gld(a.src + id[i]);
    else if (k0 + i < a.u) v[i] = gld(a.pool + slot[i]);
  }
  int tot;
  int rm = block_excl_scan(__popc(fm), sh, &tot);
  if (threadIdx.x < 64) {
    const uint32_t ex = look_back(flags, b, tag, (uint32_t)tot, a.state + GC_STATE_ERR);
    if (threadIdx.x == 0) {
      *s_ex = ex;
      if (b == a.nbu - 1) {
        istore(a.state + GC_STATE_UNION, a.u);
        istore(a.state + GC_STATE_MISSING, (int32_t)(ex + (uint32_t)tot));
      }
    }
  }
  __syncthreads();
  rm += (int)*s_ex;
  if (fm) union_probe(a.free_list, a.ftotal, ltag, fbase + rm, a.flimit, fm, slot, a.state + GC_STATE_ERR);
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    const int64_t k = k0 + i;
    if (k >= a.u) continue;
    const int32_t s = slot[i];
    gst(a.uslot + k, s);
    gst(a.packed + k, v[i]);
    if ((fm >> i) & 1u) {
      gst(a.missing + rm, id[i]);
      gst(a.mslot + rm, s);
      ++rm;
      if (s >= 0) gst(a.pool + s, v[i]);
    }
  }
}

__device__ __forceinline__ void union_data(const ReorgArgs& a, int b, const int32_t (&id)[kUItems],
                                           const int32_t (&slot)[kUItems], uint32_t fm, bool coh) {
  const int64_t k0 = (int64_t)b * kUBlock + (int64_t)threadIdx.x * kUItems;
  float4 v[kUItems];
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((fm >> i) & 1u) v[i] = gld(a.src + id[i]);
    else if (k0 + i < a.u) v[i] = coh ? ld_rec<true>(a.pool + slot[i]) : ld_rec<false>(a.pool + slot[i]);
  }
#pragma unroll
  for (int i = 0; i < kUItems; ++i) {
    const int64_t k = k0 + i;
    if (k >= a.u) continue;
    gst(a.packed + k, v[i]);
    if (((fm >> i) & 1u) && slot[i] >= 0) gst(a.pool + slot[i], v[i]);
  }
}

}  // namespace dev
}  // namespace gc
