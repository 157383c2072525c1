// Internal declarations shared by the host runtime and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gcharm.h"

namespace gc {

constexpr int kWave = 64;
constexpr int kNodeTile = 64;                           // node records per wavefront tile
constexpr int kMaxTile = 1024;                          // direct records per wavefront tile (upper bound)
constexpr int kSortMax = 8192;                          // longest per-task list sorted in LDS
constexpr int kLptChunk = 8192;                         // tasks per longest-first ordering run

// Algorithmic work per interaction (add / sub / mul = 1, fma = 2, rsqrt / rcp = 1, compare and
// select = 0), counted term by term on the implemented formulas:
//   pair or monopole, 19: d = x_j - x_i (3 sub); r^2 = d.d + eps^2 (3 fma = 6); r^-1 (rsqrt, 1);
//     m r^-1, r^-2, m r^-3 (3 mul); a += m r^-3 d (3 fma = 6).
//   quadrupole node, monopole term included, 51: d = x - com (3 sub); r^2 (3 fma = 6); r^-1 (1);
//     r^-2, r^-3, r^-5 (3 mul); S'd with S' = 3 S, stored in the node record (per component
//     1 mul + 2 fma = 5, so 15); d.S'd (1 mul + 2 fma = 5); -2.5 r^-2 (1 mul);
//     u = 1.5 T - 2.5 r^-2 d.S'd (1 fma = 2); v = r^-2 u - M (1 fma = 2); c = r^-3 v (1 mul);
//     a += c d + r^-5 S'd (6 fma = 12).  The factors 3 on S and 1.5 on T are applied once per node
//     record as it is staged, not per interaction, so they are not counted (an estimate that
//     applies them per interaction comes to about 54).
//   Lennard-Jones pair inside the cutoff, both atoms updated, 26: d = x_i - x_j - shift (the shift
//     folded into the staged source; 3 sub); r^2 (1 mul + 2 fma = 5); r^-2 (rcp, 1);
//     q = sigma^2 r^-2 (1 mul); q^3 (2 mul); f = 24 eps q^3 (2 q^3 - 1) r^-2 (1 fma + 3 mul = 5);
//     f d (3 mul); F_i += f d (3 add); F_j -= f d (3 sub).
constexpr int kFlopsPair = 19;
constexpr int kFlopsQuad = 51;
constexpr int kFlopsLJ = 26;

// ---------------------------------------------------------------- device argument blocks

struct GravArgs {
  const gc_task* tasks;
  int32_t n_tasks;
  const int2* ranges;      // direct ranges in the address space of `rec`
  const int32_t* ibeg;     // per task: first target position in `rec` (nullptr: task.i_begin)
  const int32_t* ioff;     // LISTS: per task offset into ilist
  const int32_t* joff;     // LISTS: per task offset into jlist (n_tasks + 1)
  const int32_t* ilist;
  const int32_t* jlist;
  const int32_t* node_idx;
  const float4* nodes;     // 3 float4 per node
  int32_t n_nodes;         // nodes in the table (reads past it return zero records)
  const float4* rec;       // records (packed, pool or source)
  float4* acc;             // output, by target id
  float G, eps2;
  int32_t tile;            // direct records per wavefront tile (multiple of 64)
  int32_t* queue;          // persistent schedule: work counter
  const int32_t* order;    // persistent schedule: task order
};

struct LJArgs {
  const gc_task* tasks;
  int32_t n_tasks;
  const int2* ranges;      // one range per task (j cell), address space of `rec`
  const int2* ranges_id;   // the same ranges in id space (atomic targets)
  const int32_t* ibeg;     // per task first i position (nullptr: task.i_begin)
  const float4* rec;
  float4* acc;             // force accumulators by id (F / m applied by a finishing kernel)
  const float* eps_t;
  const float* sig_t;
  int32_t n_types;
  float rc2;
  int32_t* queue;
  const int32_t* order;
  const int32_t* runs;     // runs of consecutive tasks sharing one target range: [runs[r], runs[r+1])
  int32_t n_runs;
  // gather form: target ranges (first id, count, first entry, entries) and their entries
  // (task * 2 + side; side 0: the range is the task's i range, 1: its j range)
  const int4* tgt;
  const int32_t* ent;
  int32_t n_tgt;
  const float* mass_t;     // gather form: acceleration = F / mass_t[type]
};

// ---------------------------------------------------------------- launchers (device code)

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_pool_reset(int32_t* slot_of, int32_t n_ids, uint32_t* occ, int32_t cap, hipStream_t s);
// Reorganisation state (int32 words per batch): the host reads [0, 8) after a call.
constexpr int GC_STATE_UNION = 0;    // |U|
constexpr int GC_STATE_MISSING = 1;  // records of U that were not resident
constexpr int GC_STATE_FREE = 2;     // free pool slots before the call
constexpr int GC_STATE_ERR = 4;      // nonzero: a wait hit its bound (sticky)
constexpr int GC_STATE_CHECK = 6;    // [6, 8): capacity check counts (missing, free)

struct ReorgArgs {
  const int32_t* U;        // sorted union, padded to whole union blocks
  int32_t u;
  const float4* src;       // source records by id
  const float4* staged;    // non-null: the k-th missing record (ascending id) is staged[k], copied in
                           // from the host before the launch; src is then not read
  float4* pool;
  int32_t* slot_of;
  uint32_t* occ;           // padded to whole free-scan blocks
  int32_t cap;
  int32_t pack;            // write packed[k] for every union entry
  float4* packed;
  int32_t* uslot;          // per union rank: pool slot (-1: missing and no free slot)
  int32_t* missing;        // ids of the missing records, ascending
  int32_t* mslot;          // their slots (-1: none)
  uint64_t* free_list;     // tagged free-slot entries, flimit of them
  uint64_t* ftotal;        // tagged free-slot count (null: the batch's own word in state)
  int32_t flimit;          // entries listed (0: |U|)
  int32_t* state;
  int32_t nbf, nbu;        // set by the launcher
  int32_t evict_after;     // whole-step kernel: a union block evicts what it stages at once
  int32_t list_ready;      // the free-slot list and count were completed by an earlier launch (plain
                           // loads, no waits)
};

// occupancy entries (one per slot, padded) allocated for a pool of `cap` slots
int64_t occ_words(int32_t cap);
int free_blocks(int32_t cap);
int union_blocks(int32_t u);
int64_t union_padded(int32_t u);
int32_t reorg_state_ints(int32_t u, int32_t cap);
hipError_t launch_reorg(ReorgArgs a, hipStream_t s);
hipError_t launch_gather_src(const int32_t* U, int32_t u, const float4* src, float4* packed, int32_t* state,
                             hipStream_t s);
hipError_t launch_lists(const int32_t* irank, int64_t n_i, const int32_t* jrank, int64_t n_j, const int32_t* uslot,
                        int32_t* ilist, int32_t* jlist, hipStream_t s);
hipError_t launch_count(const int32_t* U, int32_t u, const int32_t* slot_of, const uint32_t* occ, int32_t cap,
                        int32_t* out, hipStream_t s);
hipError_t launch_evict(const int32_t* ids, const int32_t* n_dev, int32_t n_bound, int32_t* slot_of, int32_t n_ids,
                        uint32_t* occ, hipStream_t s);
hipError_t launch_sort_lists(int32_t n_tasks, const int32_t* joff, int32_t* jlist, hipStream_t s);
// by_k: the k-th record is src[k] (staged from the host), else src[ids[k]]
hipError_t launch_place(const int32_t* ids, const int32_t* slots, int32_t n, const float4* src, bool by_k, float4* pool,
                        int32_t* slot_of, uint32_t* occ, hipStream_t s);
// tpl: targets per lane, 1 or 2 (each record read from LDS serves two interactions), or 3: per chunk
// of targets, whichever fills more lanes
hipError_t launch_grav(int order, bool lists, bool persistent, int tpl, const GravArgs& a, int waves_per_block,
                       int grid_blocks, hipStream_t s);
hipError_t grav_occupancy(int order, bool lists, bool persistent, int tpl, int tile, int waves_per_block, int* blocks);
// the same pass with the potential in acc.w: one workgroup per task, one target per lane, records in
// position space (not address lists)
hipError_t launch_grav_potential(int order, const GravArgs& a, int waves_per_block, hipStream_t s);
hipError_t launch_lj(bool persistent, const LJArgs& a, int waves_per_block, int grid_blocks, hipStream_t s);
// gather form: every target range's atoms written once (F / m), no atomics
hipError_t launch_lj_gather(bool persistent, const LJArgs& a, int grid_blocks, hipStream_t s);
hipError_t launch_lj_finish(float4* acc, const float* mass_t, const float4* rec_by_id, int32_t n,
                            hipStream_t s);
// *out += the tasks' in-cutoff pairs (the forward kernels' FP32 decision; self tasks i < j)
hipError_t launch_lj_count(const gc_task* tasks, int32_t n_tasks, const int2* ranges_id, const float4* rec_by_id,
                           float rc2, unsigned long long* out, hipStream_t s);

// ---------------------------------------------------------------- device-side commit

// Totals of a device commit (int64 words, zeroed before the launch).
constexpr int kDcUnion = 0, kDcDirect = 1, kDcTargets = 2, kDcMaxDirect = 3, kDcBad = 4, kDcBadTargets = 5,
              kDcMaxNode = 6, kDcTot = 8;
struct DevCommitArgs {
  gc_task* tasks;          // the batch's copy (tasks that break the contract are emptied in place)
  int32_t n_tasks;
  const int2* ranges;      // (first id, count) pairs
  int32_t n_ranges;
  const int32_t* nodes;
  int32_t n_node_refs, n_nodes;
  int32_t n_ids;
  int32_t* dc;             // per task: direct entries
  int64_t* cost;           // per task: launch-order cost
  int32_t* diff;           // 2 (n_ids + 1), zeroed: +1 / -1 at range starts / ends (all ids, target ids)
  int32_t* bs;             // 2 per id block: block sums, then their exclusive prefixes
  int32_t* ns;             // per id block: ids of U in the block, then their exclusive prefix
  int32_t* U;              // room for n_ids entries (padded to whole union blocks)
  int32_t* pos;            // n_ids: rank in U or -1
  int2* pranges;
  int32_t* pibeg, *ioff, *joff, *order;
  int64_t* tot;            // kDcTot words
};
int dc_id_blocks(int32_t n_ids);
hipError_t launch_dev_commit(const DevCommitArgs& a, hipStream_t s);
hipError_t launch_walk_tasks(int32_t b0, int32_t b1, const int32_t* bucket_node, int32_t n_nodes,
                             const int32_t* node_range, const int32_t* n_first, const int32_t* r_first, gc_task* out,
                             hipStream_t s);

// ---------------------------------------------------------------- Ewald correction

constexpr int kEwaldMaxHmax2 = 64;   // largest |h|^2 of the wave-vector sum
constexpr int kEwaldMaxH = 1056;     // half-space wave vectors with 0 < |h|^2 <= 64: 1054
struct EwaldArgs {
  const gc_task* tasks;
  int32_t n_tasks;
  const int32_t* ioff;     // per task: first target in flat order (n_tasks entries, ascending)
  int64_t n_targets;
  const int32_t* ibeg;     // per task first target position in `rec` (nullptr: task.i_begin)
  const float4* rec;
  float4* acc;             // += the correction, by target id
  float L, inv_L, alpha, GM;
  float c[3];
  int32_t nrep, hmax, hmax2;
  float kcoef;             // -2 G M / L^2
  float kdecay;            // pi^2 / (alpha L)^2
  bool quad;               // second-moment terms (S not all zero)
  float GS[6];             // G S: xx yy zz xy xz yz
  float qcoef;             // 4 pi^2 / L^4
};
hipError_t launch_ewald(const EwaldArgs& a, hipStream_t s);

// ---------------------------------------------------------------- whole-step persistent kernel

// Work items of one step, in ticket order; see step.hip.
enum { kItemFree = 1, kItemUnion = 2, kItemForce = 3 };
// One work item, by ticket (32 bytes: a block loads the next one straight into LDS while it runs
// the current one).
struct StepItem {
  int32_t kind;  // item type | round << 2
  int32_t idx;   // free-scan and union items: block index within the round's role;
                 // force items: the task's first packed target
  int32_t i_begin, i_count, j_first, j_nranges, n_first, n_count;  // force items: the task
};
static_assert(sizeof(StepItem) == 32, "StepItem is loaded as two 16-byte pieces");
struct StepRound {
  GravArgs grav;          // the round's combined pass over its packed records
  ReorgArgs reorg;        // the round's reorganisation (nbf: free-scan items, 0 after round 0; nbu)
  int32_t n_chain;        // free-slot + union items of the round
  int32_t prev;           // the latest earlier round with chain items (-1: none; kPrevFreeList: none, but
                          // the round reads round 0's free-slot list and count)
};
// An independent round (the evicting fixture): its reorganisation needs nothing of earlier rounds but
// the launch's free-slot list, which round 0's free-scan items write.
constexpr int32_t kPrevFreeList = -2;
struct StepArgs {
  const StepItem* items;  // by ticket
  int32_t n_items;
  const StepRound* rounds;
  int32_t n_rounds;
  uint64_t* ctr;          // counter c at ctr[kCtrStride * c] (all monotonic across launches); a wait that
                          // hits its bound sets the error word of its round's batch state
  uint64_t* fmeta;        // free-slot list of the launch: [0] its count, [1 + r] round r's offset into
                          // it, then the list (tagged words, tag = launch epoch + 1)
  uint32_t spin_limit;    // probes after which a wait gives up and sets its round's error word
  int32_t fail_round;     // test hook: this round's force items wait for one data part too many (-1: none)
  uint32_t fail_spins;    // and give up after this many probes
  int32_t has_force;      // the launch runs the force items (0: reorganisation items only)
};
// Dependencies complete within microseconds; the default bound (about a second) only keeps a broken
// state from holding the grid.
constexpr uint32_t kStepSpinLimit = 1u << 20;
constexpr int kCtrStride = 32;  // one 256-byte line per step counter
constexpr int kCtrTickets = 0, kCtrExits = 1, kCtrEpoch = 2, kCtrRounds = 3;  // then per round r:
                                // kCtrRounds + 2r table parts (free-scan and union items) done,
                                // + 1 data parts (union items) done
constexpr int kStepLead = 3;    // rounds by which the reorganisation items precede the passes
hipError_t launch_step(int order, int tpl, const StepArgs& a, int grid, int tile, hipStream_t s);
// the same schedule with reorganisation items only (a.has_force = 0), in a kernel without force code
hipError_t launch_step_reorg(const StepArgs& a, int grid, hipStream_t s);
// The combined pass over the tasks of several rounds in one launch: items[b] (kind = round index,
// idx = first packed target) with rounds[kind]; waves_per_block waves per task.
hipError_t launch_grav_rounds(int order, int tpl, const StepItem* items, int32_t n_items, const GravArgs* rounds,
                              int tile, int waves_per_block, hipStream_t s);
hipError_t step_occupancy(int order, int tpl, int tile, int* blocks);

struct GravAdjArgs {
  GravArgs f;              // forward arguments (lists, records, nodes)
  const float4* cot;       // by id
  float4* gpos;            // by id
  float* gmass;            // by id
  const int32_t* src_id;   // position in rec -> id (PACK: U; LISTS: slot -> id map; nullptr: identity)
  const int32_t* joff;     // per task: first direct visit (the task's flat direct positions follow in order)
  float4* vnode;           // per node visit (entry of the node lists): dL/dcom (3) and dL/dM; quadrupole:
                           // then sym(dL/dS) xx yy zz xy xz yz and two unused floats (3 float4 per visit)
  float4* vdir;            // per direct visit: dL/dx (3) and dL/dm of the source
};
// Visits of one node are summed in chunks of at most this many (one wavefront per chunk), so that a
// node found in nearly every task's list adds no long serial tail.
constexpr int kVisitChunk = 256;
// order 1: monopole nodes (one float4 per node visit); order 2: quadrupole nodes (three)
hipError_t launch_grav_adjoint(bool packed, int order, const GravAdjArgs& a, int waves_per_block, hipStream_t s);
// The gradients of the visits, gathered through the visit indices built on the host: node visits
// summed per chunk into `part` (chunks of each node contiguous, chunk_first per node), then per node
// and pushed to the member particles; direct visits, sorted by source id (dkey), summed per id in
// runs of a wavefront and added to gpos / gmass.
hipError_t launch_visit_sums(int order, const float4* vnode, const int32_t* nvis, const int2* chunks,
                             int32_t n_chunks, float4* part, hipStream_t s);
// Nodes whose (first id, count) range is not inside [0, n_ids) are skipped and counted in *bad.
hipError_t launch_node_chain(int order, const int32_t* node_range, int32_t n_nodes, const float4* nodes,
                             const float4* part, const int32_t* chunk_first, const float4* rec_by_id, int32_t n_ids,
                             float4* gpos, float* gmass, int32_t* bad, hipStream_t s);
hipError_t launch_direct_sums(const float4* vdir, const int32_t* dvis, const int32_t* dkey, int32_t n_vis,
                              float4* gpos, float* gmass, hipStream_t s);
struct LJAdjArgs {
  LJArgs f;
  const float4* cot;       // by id
  const float* mass_t;
  float4* gpos;
  float* gparam;           // 2 * n_types
  float4* force;           // forward forces by id (for the mass gradient)
  float* ppart;            // per block: 2 n_types^2 partial parameter derivatives (lj_adjoint_blocks rows)
};
int lj_adjoint_blocks(const LJArgs& f, bool gather);
hipError_t launch_lj_adjoint(const LJAdjArgs& a, int waves_per_block, hipStream_t s);
hipError_t launch_lj_adjoint_gather(const LJAdjArgs& a, hipStream_t s);
hipError_t launch_lj_mass_grad(const float4* cot, const float4* force, const float* mass_t,
                               const float4* rec_by_id, float* gmass, int32_t n, hipStream_t s);

}  // namespace gc
