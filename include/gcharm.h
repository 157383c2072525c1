/*
 * gcharm.h: C ABI of the combined irregular-task force library for MI355X
 * (gfx950).
 *
 * The library runs many small, uneven work requests (tasks) in one device
 * launch, after a data-reorganisation pass that reuses records already
 * resident in a device pool, stages only the missing ones, and packs the union
 * of what a combined request touches into one contiguous buffer.  The
 * operations follow the paper's runtime strategies:
 *   - a work request names the data it touches (Sec. 3.2: a workRequest holds
 *     the indices of the chare buffers it reads);
 *   - the runtime keeps a chare table mapping resident data to device slots
 *     and transfers only data not already on the device (Sec. 2.2, Sec. 3.2);
 *   - accessed indices are kept sorted so that threads read in index order
 *     (Sec. 3.2, reassignment by sorted indices; data reorganisation named as
 *     the alternative);
 *   - many requests are combined into one kernel (Sec. 2.2, Sec. 3.1).
 *
 * Conventions for every entry point:
 *   - Every call returns gc_status; 0 is success.  No exception or abort
 *     crosses the ABI.  On failure gc_last_error(ctx) holds a message that
 *     stays valid until the next call on that context.
 *   - "host" arrays are read during the call only (copied); "device" arrays
 *     are device-resident (hipMalloc / torch) and owned by the caller.
 *   - Streams are hipStream_t passed as void* (NULL = default stream); the
 *     library enqueues work and returns without synchronising unless a call
 *     says otherwise.
 *   - Records are 16 bytes: float4 (x, y, z, m) for gravity, float4
 *     (x, y, z, type) for Lennard-Jones (type stored as a float 0.0, 1.0, ...).
 *   - A context is single-threaded: calls on one context (and on pools and
 *     batches created from it) must not overlap from different host threads.
 *   - After an asynchronous device error a context is poisoned: the call that
 *     observes it returns GC_E_HIP and every later call GC_E_STATE, until
 *     gc_finalize.
 */
#ifndef GCHARM_H
#define GCHARM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GC_OK = 0,
  GC_E_INVAL = 1,       /* bad argument: ids or ranges out of bounds, bad mode, NULL pointer */
  GC_E_NOMEM = 2,       /* device or pinned allocation failed */
  GC_E_FULL = 3,        /* the pool has fewer free slots than missing records */
  GC_E_STATE = 4,       /* call out of order, or context poisoned */
  GC_E_HIP = 5,         /* a HIP runtime call or kernel failed */
  GC_E_UNSUPPORTED = 6  /* combination not implemented */
} gc_status;

typedef struct gc_ctx_* gc_ctx;
typedef struct gc_pool_* gc_pool;
typedef struct gc_batch_* gc_batch;
typedef struct gc_graph_* gc_graph;

/* ---------------------------------------------------------------- context */

/*
 * The caller's device allocator.  alloc_fn returns `bytes` of device memory of
 * device `device` (aligned to at least 256 bytes) or NULL; free_fn takes back a
 * pointer alloc_fn returned.  Both receive the `user` pointer given to gc_init.
 * They are called from the host thread that makes the library call (never
 * during graph capture), and free_fn only after the device is idle, so a
 * stream-ordered caching allocator (torch's) may reuse the memory at once.
 */
typedef void* (*gc_alloc_fn)(size_t bytes, void* user);
typedef void (*gc_free_fn)(void* ptr, void* user);

/* Open a context on HIP device `device` (makes it current for the calling thread).
 * Every device buffer the library owns (pool records and chare table, batch
 * buffers, graph and list-walk scratch) is taken from alloc_fn / free_fn;
 * both NULL: hipMalloc / hipFree (one NULL and not the other: GC_E_INVAL).
 * A context and everything made from it are used from one host thread at a
 * time: calls on one context must not overlap (the context holds the last
 * error and the list walk's scratch). */
gc_status gc_init(int device, gc_alloc_fn alloc_fn, gc_free_fn free_fn, void* user, gc_ctx* out);
/* Release everything the context owns (pools and batches must be destroyed first or are leaked). */
gc_status gc_finalize(gc_ctx ctx);
/* Last error message of the context ("" if none). Owned by the context. */
const char* gc_last_error(gc_ctx ctx);
/* Library version string, static. */
const char* gc_version(void);

/*
 * Test hook: the next call on `ctx` that reaches the device-error check
 * behaves as if an asynchronous device error with HIP code `hip_error` (!= 0)
 * had surfaced: it returns GC_E_HIP and poisons the context.  Host state only;
 * nothing is sent to the device.
 */
gc_status gc_debug_inject_error(gc_ctx ctx, int hip_error);

/* ---------------------------------------------------------------- pool (chare table) */

/*
 * A device pool of `capacity` 16-byte record slots plus the chare table
 * slot_of[n_ids] (int32, -1 = not resident) over ids [0, n_ids) (Sec. 3.2:
 * the chare table maps chare buffers to device slots).  All slots start free.
 * Pool memory is owned by the library.
 */
gc_status gc_pool_create(gc_ctx ctx, int32_t n_ids, int32_t capacity, gc_pool* out);
gc_status gc_pool_destroy(gc_pool pool);

/*
 * Where records of ids not resident are read from when a reorganisation
 * stages them (Sec. 3.2: only data not already on the device is moved).
 * `records` holds n_ids float4 records indexed by id.  It may be device
 * memory (staging is then a device gather) or pinned host memory from
 * hipHostMalloc (staging then reads it over PCIe from the kernel; only the
 * missing records cross the link).  The caller owns it; it must stay valid
 * and unchanged while batches reorganised against this pool are in flight.
 */
gc_status gc_pool_set_source(gc_pool pool, const void* records);

/*
 * Host source with staging copies (Sec. 2.2: the runtime copies to the
 * device only the data a request needs that is not already there; Sec. 3.2:
 * the chare table tells the runtime which buffers are resident).  `records`
 * holds n_ids float4 records by id in ordinary host memory (pageable or
 * pinned), caller-owned; it is read only during gc_pool_place and
 * gc_reorganize calls, never afterwards.  Replaces a source set by
 * gc_pool_set_source.  The pool then keeps a host mirror of its chare table,
 * updated by every call in call order with the device's own allocation rule
 * (the k-th missing id takes the k-th lowest free slot), so a reorganisation
 * knows its missing records without reading the device; the host packs them
 * into a pinned staging buffer that gc_reorganize copies in on its side
 * stream.  The mirror is read back from the device once (synchronising) when
 * the device changed the table without the host (a reorganisation from a
 * device source, a graph launch, a place or evict issued before the host
 * source was set).  Such a pool cannot be captured in a graph
 * (GC_E_UNSUPPORTED), and NONE reorganisations, Lennard-Jones passes and
 * backward calls need a device source.
 */
gc_status gc_pool_set_host_source(gc_pool pool, const void* records);

/*
 * The host mirror of a host-source pool's chare table (n_ids int32, -1 = not
 * resident) copied to slot_of_host; equals gc_pool_query once the device has
 * run every call made so far.  GC_E_STATE without a host source.
 */
gc_status gc_pool_query_mirror(gc_pool pool, int32_t* slot_of_host, void* stream);

/*
 * Residency fixture: make ids[k] resident in slots[k] (device int32 arrays of
 * length n), copying their records from the source.  Ids must be distinct,
 * not yet resident, and slots distinct and free; violations are not detected
 * on the device (the host does not see the arrays) and leave the table
 * inconsistent.  Asynchronous on `stream`, except with a host source: the
 * host then reads ids and slots (synchronising `stream`), rejects ids or
 * slots out of range with GC_E_INVAL, and copies the records in.
 */
gc_status gc_pool_place(gc_pool pool, const int32_t* ids_dev, const int32_t* slots_dev, int32_t n, void* stream);

/* Evict every record (all slots free, slot_of all -1). Asynchronous. */
gc_status gc_pool_reset(gc_pool pool, void* stream);

/*
 * Evict ids_dev[0, n) (device int32): each resident id leaves the table and
 * its slot becomes free; ids outside [0, n_ids) or not resident are skipped.
 * The record data stay in the slot until a later staging overwrites them.
 * Asynchronous on `stream` (a host-source pool with a current mirror reads
 * the ids first, synchronising `stream`).
 */
gc_status gc_pool_evict(gc_pool pool, const int32_t* ids_dev, int32_t n, void* stream);

/*
 * Evict the records that the last reorganisation of `batch` (PACK, INDIRECT
 * or SORTED, against this pool) staged, i.e. its missing list; the count is
 * read on the device, so the call is graph-capture safe and never
 * synchronises.  A no-op after REDUNDANT or NONE or before any
 * reorganisation of the batch; GC_E_STATE if the batch was last reorganised
 * against another pool.  Used to keep a pool at a
 * base residency across rounds (staged data treated as transient).
 */
gc_status gc_pool_evict_staged(gc_pool pool, gc_batch batch, void* stream);

/* Copy slot_of (n_ids int32) to host memory; synchronises `stream`. */
gc_status gc_pool_query(gc_pool pool, int32_t* slot_of_host, void* stream);

/* Device pointers of the pool internals (float4 records[capacity], int32 slot_of[n_ids]). */
gc_status gc_pool_device_ptrs(gc_pool pool, void** records, int32_t** slot_of);

/* ---------------------------------------------------------------- batch (combined request) */

enum { GC_KIND_GRAV = 0, GC_KIND_LJ = 1 };
enum { GC_TASK_SELF = 1 };  /* LJ: i and j ranges are the same cell; pairs i < j only */

/*
 * One work request (Sec. 2.2: a workRequest; Sec. 4.1: a bucket whose
 * particles share one interaction list; Sec. 4.2: a compute object for a
 * pair of patches).
 *   i_begin, i_count   target ids [i_begin, i_begin + i_count)
 *   j_first, j_nranges direct source ranges: pairs (begin, count) at
 *                      j_ranges[2*j_first ...] of the same submit call
 *   n_first, n_count   node references node_idx[n_first ...] of the same call
 *                      (gravity only)
 *   flags              GC_TASK_SELF (Lennard-Jones)
 *   shift              Lennard-Jones periodic image shift of the j range
 *                      (the j atoms' images sit at x_j + shift); 0 for gravity
 * Gravity: targets need not lie inside the direct ranges; a target id found in
 * its own direct ranges contributes nothing (j == i is skipped).
 * Lennard-Jones: exactly one j range per task.
 */
typedef struct {
  int32_t i_begin, i_count;
  int32_t j_first, j_nranges;
  int32_t n_first, n_count;
  int32_t flags;
  float shift[3];
} gc_task;

/* A batch of kind GC_KIND_GRAV or GC_KIND_LJ over ids [0, n_ids). */
gc_status gc_batch_create(gc_ctx ctx, int32_t kind, int32_t n_ids, gc_batch* out);
gc_status gc_batch_destroy(gc_batch batch);
/* Drop all submitted tasks (device buffers are kept for reuse). */
gc_status gc_batch_reset(gc_batch batch);

/*
 * Append n_tasks tasks (host arrays, copied).  j_ranges holds n_ranges
 * (begin, count) pairs; node_idx holds n_node_refs node indices; tasks index
 * into these arrays relative to this call.  Validation (host side, strong
 * guarantee: on error nothing is appended): ids and ranges inside [0, n_ids),
 * counts >= 0, list slices inside the given arrays, node indices >= 0 (and
 * below the node table's size, checked where the table is given),
 * no two nonempty direct ranges of one task overlapping (a source listed
 * twice would be summed twice), Lennard-Jones tasks with exactly one j range
 * and no nodes.
 */
gc_status gc_submit_tasks(gc_batch batch, const gc_task* tasks, int32_t n_tasks, const int32_t* j_ranges,
                          int32_t n_ranges, const int32_t* node_idx, int32_t n_node_refs);

/*
 * Fix the batch (once; later calls are no-ops until the next submit or
 * reset): the union U of the batch, i.e. the ids of every target and direct
 * range, ascending and without duplicates (Sec. 3.2: the runtime keeps the
 * request's indices sorted as they are inserted), together with each range's
 * and each task's first position in U (a range is contiguous in U), the
 * per-task offsets and the launch order (longest first within runs of 8,192
 * tasks).  Host submissions: built on the host and uploaded with the tasks.
 * Device submissions: built on the device (U by marking every range in a
 * difference array and two prefix sums, so ids are never sorted), with only
 * eight totals read back.  Synchronises `stream` in both cases.  Later calls
 * that need the lists on the host (gc_batch_maps, address-list modes, host
 * staging, gc_backward, gc_graph_capture) copy them from the device once.
 */
gc_status gc_batch_commit(gc_batch batch, void* stream);

/*
 * Device-side submission (gravity batches): the request's tasks, ranges and
 * node references are already in device memory -- typically the list walk's
 * output (gc_tree_walk, gc_walk_tasks) -- in the layout of gc_submit_tasks
 * (task slices relative to the given arrays).  The batch copies them device
 * to device on `stream`; nothing is read on the host.  The batch must hold no
 * other submission (GC_E_STATE: reset it first), and gc_submit_tasks is
 * refused until the next reset.  Validation moves to gc_batch_commit, which
 * then runs on the device: ids, counts and slices in bounds, each task's
 * direct ranges in ascending id order and disjoint (as the walk emits them),
 * node indices in [0, n_nodes), no id targeted by two tasks, no flags or
 * shift.  A batch that breaks it is reported by gc_batch_commit with
 * GC_E_INVAL and stays uncommitted.
 */
gc_status gc_submit_tasks_device(gc_batch batch, const gc_task* tasks_dev, int32_t n_tasks,
                                 const int32_t* j_ranges_dev, int32_t n_ranges, const int32_t* node_idx_dev,
                                 int32_t n_node_refs, int32_t n_nodes, void* stream);

/*
 * The tasks of buckets [b0, b1) (0 <= b0 <= b1 <= n_buckets, the walk's
 * bucket count) of a list walk, written to tasks_dev (device,
 * b1 - b0 gc_task records; Sec. 4.1: a bucket's particles form one work
 * request that shares the bucket's lists): bucket b's targets are its leaf's
 * id range (node_range_dev, int32 pairs (first id, count) per node), its
 * direct ranges r_first_dev[b] .. r_first_dev[b + 1] and node references
 * n_first_dev[b] .. n_first_dev[b + 1] of the walk's output, numbered from
 * those of bucket b0, so that the walk's ranges_dev + 2 * r_first[b0] and
 * node_idx_dev + n_first[b0] are the arrays to submit with them.  A leaf
 * index outside [0, n_nodes) gives a task that gc_batch_commit refuses.
 * Asynchronous on `stream`.
 */
gc_status gc_walk_tasks(gc_ctx ctx, int32_t n_buckets, int32_t b0, int32_t b1, const int32_t* bucket_node_dev,
                        int32_t n_nodes,
                        const int32_t* node_range_dev, const int32_t* n_first_dev, const int32_t* r_first_dev,
                        gc_task* tasks_dev, void* stream);

/* Number of tasks, ranges, node refs, direct entries (sum of range counts) and targets. */
gc_status gc_batch_sizes(gc_batch batch, int64_t* out5);

/*
 * Device-side error words of a batch, read after waiting on `stream`:
 * GC_E_HIP if a bounded wait of one of its reorganisations (per-batch or
 * whole-step) gave up since the reorganisation state was last cleared (at
 * the first reorganisation after a commit, and at graph capture): its maps
 * and the forces of the pass that read them are then unspecified;
 * GC_E_INVAL if a backward call met node ranges outside [0, n_ids) (those
 * nodes' gradients were not pushed to members; sticky until the next
 * commit); else GC_OK.  The context is not poisoned.
 */
gc_status gc_batch_status(gc_batch batch, void* stream);

/*
 * Reorganisation (Sec. 3.2) of a committed batch against a pool, on `stream`:
 *  a. U and pos[id] = rank in U are those fixed at commit;
 *  b. missing = ids of U not resident, ascending (chare-table lookup);
 *  c. the k-th missing id gets the k-th lowest free slot; its record is copied
 *     from the pool's source into that slot (it stays resident afterwards);
 *     steps b and c and the PACK gather run as one kernel launch;
 *  d. then, by mode:
 *   GC_REORG_PACK      packed[k] = pool[slot_of[U[k]]] for k < |U|; every
 *                      range (b, c) becomes (pos[b], c) and targets read
 *                      packed[pos[i]]: contiguous, coalesced reads;
 *   GC_REORG_INDIRECT  per task, the pool slot of every target and of every
 *                      direct id in list order (the per-request address
 *                      buffer; two dependent loads per record);
 *   GC_REORG_SORTED    as INDIRECT with each task's direct slots sorted
 *                      ascending (reassignment by sorted indices);
 *   GC_REORG_REDUNDANT no reuse: every id of U is copied from the source into
 *                      packed (redundant transfer, fully coalesced); the pool
 *                      is not touched;
 *   GC_REORG_NONE      no reorganisation: the source must be device memory
 *                      and is read in place by id.
 * With check_capacity != 0 the missing and free counts are taken first and
 * GC_E_FULL is returned (pool unchanged) if the pool lacks free slots; this
 * synchronises the stream.  With check_capacity = 0 the call never
 * synchronises; a missing record left without a slot is then still packed
 * from the source (PACK), gets slot 0 in address lists, is not made
 * resident, and gc_batch_maps reports GC_E_FULL.  Reorganisations of
 * batches sharing a pool must not run concurrently: issue them on one
 * `stream`.
 * Host source (gc_pool_set_host_source; Sec. 2.2, Sec. 3.2: host-issued
 * copies of only the missing data): the host takes the missing ids from its
 * mirror of the chare table, packs their records into the batch's pinned
 * staging buffer (REDUNDANT: every record of U) and copies them to the device
 * on `side_stream` (NULL: on `stream`); the kernel on `stream` waits for the
 * copy, and the copy waits only for the work on `stream` that last read this
 * batch's staged or packed records, so it overlaps the passes of other
 * batches.  The capacity check then uses the mirror and does not
 * synchronise.  The call blocks the host only while the batch's previous
 * copy is still running (its pinned buffer is reused).  With a device
 * source `side_stream` is not used.
 */
enum { GC_REORG_REDUNDANT = 0, GC_REORG_INDIRECT = 1, GC_REORG_SORTED = 2, GC_REORG_PACK = 3, GC_REORG_NONE = 4 };
gc_status gc_reorganize(gc_batch batch, gc_pool pool, int32_t mode, int32_t check_capacity, void* stream,
                        void* side_stream);

/*
 * Host copies of the last reorganisation's maps (synchronises `stream`):
 * counts[0] = |U|, counts[1] = #missing.  Each output may be NULL.
 *   U[|U|], pos[n_ids] (-1 outside U), missing[#missing],
 *   new_slot[#missing] (slot given to missing[k]; REDUNDANT: not written),
 *   pranges[2*n_ranges], pi_begin[n_tasks] (PACK / REDUNDANT),
 *   ilist[sum i_count], jlist[sum direct entries] (INDIRECT / SORTED).
 * Sizes are from gc_batch_sizes.
 */
gc_status gc_batch_maps(gc_batch batch, int64_t* counts, int32_t* U, int32_t* pos, int32_t* missing,
                        int32_t* new_slot, int32_t* pranges, int32_t* pi_begin, int32_t* ilist, int32_t* jlist,
                        void* stream);

/* ---------------------------------------------------------------- combined force pass */

enum { GC_FORCE_GRAV_MONO = 1, GC_FORCE_GRAV_QUAD = 2, GC_FORCE_LJ = 3 };

/*
 * Force-law parameters.
 * Gravity (Sec. 4.1 workload; softened Newtonian gravity with Barnes-Hut
 * node terms): G, soft_eps > 0 (Plummer softening); node records are 12
 * floats (com x y z, M, Sxx Syy Szz Sxy, Sxz Syz T, 0) with S the raw second
 * moment about the centre of mass and T its trace; GC_FORCE_GRAV_MONO reads
 * only the first 4 floats of each node record.
 *   direct:     a_i += G m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^{3/2}, j != i
 *   monopole:   a_i += -G M d / r^3, d = x_i - com, r^2 = |d|^2 + eps^2
 *   quadrupole: a_i += G [3 S d / r^5 - 15/2 (d.S.d) d / r^7 + 3/2 T d / r^5]
 * Lennard-Jones (Sec. 4.2 workload; a compute object updates the forces of
 * both cells): per-type eps_t, sig_t, mass_t (device float arrays of n_types),
 * Lorentz-Berthelot mixing, cutoff r_cut (pairs with r^2 < r_cut^2, decided
 * in FP32), force on i = 24 eps (2 q^6 - q^3) / r^2 d, q = sigma^2 / r^2,
 * d = x_i - x_j - shift, equal and opposite on j; a = F / m.
 */
/*
 * Schedules.  GC_SCHED_TASKS: one launch, one workgroup per task, longest
 * tasks first.  GC_SCHED_QUEUE: a persistent grid (CUs x occupancy) takes
 * tasks from a device counter in the same order.  GC_SCHED_STEP (graph
 * capture only, gravity, PACK, one pool, fixture NONE or EVICT_STAGED,
 * distinct batches): one persistent launch runs all captured steps -- each
 * step's reorganisation (with the evicting fixture, the eviction of what it
 * stages) and combined pass -- as ordered work items with device-side
 * dependencies, the reorganisation three steps ahead of the passes; the
 * free-slot scan runs once per launch (later steps take the free slots after
 * those kept by earlier ones); 4 waves per task; results bitwise equal to the
 * per-step launches.  With the evicting fixture a small kernel ahead of the
 * launch evicts what the last step left staged before it.
 * GC_SCHED_ROUNDS (graph capture only, same conditions as GC_SCHED_STEP):
 * the captured steps' reorganisations run as the work items of one
 * persistent launch (with the evicting fixture side by side, each step seeing
 * the pool as the first found it; otherwise in a chain), then one combined
 * launch runs every task of every step from its step's packed records
 * (Sec. 3.1: all of the combined requests in one kernel), tasks in each
 * step's launch order, steps in order, waves_per_block waves per task;
 * results bitwise equal to the per-step launches of the same shape.
 */
enum { GC_SCHED_TASKS = 0, GC_SCHED_QUEUE = 1, GC_SCHED_STEP = 2, GC_SCHED_ROUNDS = 3 };

typedef struct {
  int32_t kind;             /* GC_FORCE_* */
  float G, soft_eps;        /* gravity */
  int32_t n_types;          /* Lennard-Jones */
  const float* eps_t;       /* device */
  const float* sig_t;       /* device */
  const float* mass_t;      /* device */
  float r_cut;
  int32_t schedule;         /* GC_SCHED_*: how the combined pass is launched */
  int32_t tile;             /* direct-record tile per wavefront: 0 = default (256); 64..1024, multiple of 64 */
  int32_t waves_per_block;  /* 0 = default (4); 1..8 */
  int32_t grid_blocks;      /* persistent schedule: 0 = CUs x occupancy */
  int32_t targets_per_lane; /* gravity: 0 or 1 = one target per lane; 2 = each lane
                               holds two targets of its task, so every record read
                               from LDS serves two interactions; 3 = per chunk of n
                               <= 64 targets, two where floor(64 / ceil(n / 2)) >
                               2 floor(64 / n) (more lanes busy), else one.  The
                               modes split the sources over different slices, so
                               they agree to rounding; each gives the same bits on
                               every launch, schedule and aggregation */
  int32_t n_nodes;          /* gravity: node records in nodes_dev; every node index the
                               batch holds must be below it (GC_E_INVAL otherwise);
                               at most 2^24 nodes, and fewer than 2^28 direct records
                               per task (GC_E_UNSUPPORTED otherwise) */
  int32_t want_potential;   /* gravity, 1: also write in acc.w the potential of the
                               target's terms, phi_i = -G [sum over its direct sources
                               j != i of m_j / (|x_j - x_i|^2 + eps^2)^{1/2} + sum over
                               its nodes of M/r + 3/2 d.S.d / r^5 - T / (2 r^3)], the
                               function whose negative gradient is the acceleration
                               (one workgroup per task and one target per lane: the
                               schedule and targets_per_lane fields are not used);
                               GC_E_UNSUPPORTED for Lennard-Jones, address-list modes
                               and the whole-step schedule */
  int32_t deterministic;    /* 1: results must be the same bits on every call; a path
                               that sums with atomics then returns GC_E_UNSUPPORTED */
  int32_t aggregation;      /* gravity: tasks combined per launch (Sec. 3.1: how many
                               work requests one kernel takes); 0 = all tasks of the
                               batch in one launch, k > 0 = consecutive launches of k
                               tasks each in the batch's launch order (same results) */
} gc_force_params;

/*
 * The combined kernel (Sec. 3.1: many requests, one launch): every task of a
 * reorganised batch computes its targets' accelerations; acc_dev is float4
 * [n_ids] (x, y, z acceleration, w = 0), caller-owned.  Gravity writes the
 * rows of targeted ids only (each id must be the target of at most one
 * task).  Lennard-Jones writes every row (zero for ids no task touches).  When
 * any two target ranges of the batch (the tasks' i ranges and the j ranges of
 * the tasks that are not self tasks) are equal or disjoint, as for cell tasks,
 * one wavefront per range sums its atoms' forces from every task on either
 * side and writes them once: no atomics, the same bits on every launch;
 * otherwise the forces of both sides are accumulated with FP32 atomics.
 * nodes_dev: float [n_nodes * 12] (gravity), unused for Lennard-Jones.
 * Asynchronous.
 */
gc_status gc_launch_combined(gc_batch batch, const gc_force_params* prm, const float* nodes_dev, float* acc_dev,
                             void* stream);

/* Fill n floats with 0 by a kernel (graph-capture safe). */
gc_status gc_zero_f32(gc_ctx ctx, float* dev, int64_t n, void* stream);

/* ---------------------------------------------------------------- adjoint */

/*
 * Vector-Jacobian product of L = sum_i cot_i . a_i for the last combined pass
 * of `batch` (same reorganisation, same parameters), recomputing pair terms.
 *   cot_dev   float4 [n_ids] cotangent on acc (w ignored)
 *   gpos_dev  float4 [n_ids] += dL/dx (w unused), caller zeroes first
 *   gmass_dev float  [n_ids] += dL/dm (gravity: source masses and node mass
 *             chain; Lennard-Jones: per-atom mass as if each atom had its own)
 *   gparam_dev float [2 * n_types] += (dL/deps_t, dL/dsig_t) (Lennard-Jones)
 * Gravity supports GC_FORCE_GRAV_MONO and GC_FORCE_GRAV_QUAD; node gradients
 * flow to member particles through com = sum m_k x_k / M, M = sum m_k and,
 * with quadrupoles, S = sum m_k (x_k - com)(x_k - com)^T (node_range_dev: int32
 * [2 * n_nodes] (first id, count) of each node's members; members are read
 * in place from the pool's source, which must be device memory).  Lists and
 * cutoff decisions are those of the forward pass.  Gravity keeps each task's
 * gradient for each node-list entry and each direct source in a record of its
 * own and sums the records per node and per particle in a fixed order; the
 * first gravity call on a batch (and any call with another n_nodes) builds the
 * node -> entries and particle -> entries indices on the host and uploads them,
 * waiting on `stream` (GC_E_INVAL if a node index is >= n_nodes).  The batch
 * then holds 52 bytes per node-list entry, 24 per direct source entry and a
 * few bytes per node until it is destroyed.  Otherwise asynchronous.
 */
gc_status gc_backward(gc_batch batch, const gc_force_params* prm, const float* nodes_dev,
                      const int32_t* node_range_dev, int32_t n_nodes, const float* cot_dev, float* gpos_dev,
                      float* gmass_dev, float* gparam_dev, void* stream);

/* ---------------------------------------------------------------- interaction lists */

/*
 * Barnes-Hut interaction lists of every bucket's work request (Sec. 4.1: the
 * particles of a bucket share one node list and one direct list), built on the
 * device.  Tree contract: nodes numbered in pre-order, children in ascending
 * index, every node's ids contiguous (node_range_dev: int32 [2 * n_nodes]
 * (first id, count), count >= 1); node_com_dev: double [3 * n_nodes] centres of
 * mass; node_side_dev: double [n_nodes] cube sides; rec_dev: float4 [n_ids]
 * (x, y, z, m); bucket_node_dev: int32 [n_buckets], each bucket's leaf.
 * Opening test, in FP64 with correctly rounded operations: bucket B takes node
 * N when theta > 0, N's id range does not overlap B's and side(N) < theta *
 * dist(com(N), box(B)), box(B) the tight bounding box of B's positions, dist
 * from (e_x^2 + e_y^2) + e_z^2 with e the per-axis distance outside the box;
 * a leaf that is not taken goes to the direct list as its id range, any other
 * node is opened.  Lists follow the descent order (children ascending).
 * Outputs (device, caller-owned): n_first_dev / r_first_dev int32
 * [n_buckets + 1] offsets into node_idx_dev (int32 [node_cap]) and ranges_dev
 * (int32 [2 * range_cap], (first id, count) pairs); totals (host) receives the
 * node-entry and range totals.  GC_E_FULL when a capacity is short (offsets
 * and totals are then set, the lists not written: call again with room);
 * GC_E_INVAL for a bucket whose leaf index or id range is out of bounds.  The
 * call waits on `stream` (twice: for the totals and at the end).  The context
 * keeps room for up to 2,048 node entries and 128 ranges per bucket (9 KB per
 * bucket of the largest call) until gc_finalize; a bucket with more is walked
 * twice.
 */
gc_status gc_tree_walk(gc_ctx ctx, int32_t n_nodes, const int32_t* node_range_dev, const double* node_com_dev,
                       const double* node_side_dev, const float* rec_dev, int32_t n_ids, int32_t n_buckets,
                       const int32_t* bucket_node_dev, double theta, int32_t* n_first_dev, int32_t* r_first_dev,
                       int32_t* node_idx_dev, int64_t node_cap, int32_t* ranges_dev, int64_t range_cap,
                       int64_t* totals, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the walk of
 * gc_tree_walk, with the same arguments, outputs, errors and results, that
 * allocates nothing.  Its scratch (the subtree ends of the nodes, 4 bytes
 * each, and the totals) lives in one fixed device array of the library,
 * 8 MiB + 256 bytes, which each device holds until the process ends: trees of
 * at most 2^21 nodes (GC_E_INVAL beyond).  It keeps no per-bucket room, so
 * every bucket is walked twice (count, then fill).  Every call on a device
 * shares that device's array, which keeps the last call's contents (the
 * totals are cleared by a kernel at the start of each call): calls that
 * overlap on one device race, whatever their contexts.  Waits on `stream`
 * like gc_tree_walk.
 */
gc_status gc_tree_walk_noalloc(gc_ctx ctx, int32_t n_nodes, const int32_t* node_range_dev, const double* node_com_dev,
                               const double* node_side_dev, const float* rec_dev, int32_t n_ids, int32_t n_buckets,
                               const int32_t* bucket_node_dev, double theta, int32_t* n_first_dev,
                               int32_t* r_first_dev, int32_t* node_idx_dev, int64_t node_cap, int32_t* ranges_dev,
                               int64_t range_cap, int64_t* totals, void* stream);

/* ---------------------------------------------------------------- graphs */

/*
 * Capture a sequence of (reorganise, combined pass) steps over several
 * batches into one HIP graph on `stream` and instantiate it.  Each step k:
 * an optional residency fixture, gc_reorganize(batches[k], pools[k],
 * modes[k], check_capacity = 0), then gc_launch_combined(batches[k], prm,
 * nodes_dev, acc_dev).  Batches must be committed; their reorganisation
 * state is cleared once at capture.  Fixtures:
 *   GC_FIXTURE_NONE          residency carries over from step to step;
 *   GC_FIXTURE_RESET_PLACE   each pool is reset before its step and the
 *                            placements place_ids/place_slots/place_n of
 *                            that step are applied (every replay starts
 *                            from the same residency);
 *   GC_FIXTURE_EVICT_STAGED  before step k the records staged by step k-1
 *                            (cyclically: step 0 evicts those of the last
 *                            step of the previous replay) are evicted, so a
 *                            base residency set up by the caller holds at
 *                            every step (one pool for all steps).
 * When every step uses PACK, REDUNDANT or NONE and no batch appears twice,
 * each step's combined pass reads only its own batch's buffers, so it is
 * placed on a side stream and overlaps the following steps' reorganisations
 * and passes (the pool-touching chain stays in order); otherwise the steps
 * run strictly in sequence.  The graph owns its side streams.
 */
enum { GC_FIXTURE_NONE = 0, GC_FIXTURE_RESET_PLACE = 1, GC_FIXTURE_EVICT_STAGED = 2 };
gc_status gc_graph_capture(gc_ctx ctx, int32_t n_steps, gc_batch* batches, gc_pool* pools, const int32_t* modes,
                           const gc_force_params* prm, const float* nodes_dev, float* acc_dev, int32_t fixture,
                           const int32_t* const* place_ids, const int32_t* const* place_slots,
                           const int32_t* place_n, void* stream, gc_graph* out);
gc_status gc_graph_launch(gc_graph graph, void* stream);
gc_status gc_graph_destroy(gc_graph graph);

/*
 * Waits on `stream`, then reads the error words of every batch the graph
 * reorganises: GC_E_HIP if a bounded wait of a reorganisation, or of the
 * whole-step schedule's dependencies, gave up in any launch since capture
 * (the results of those launches are unspecified), else GC_OK.  The words
 * are sticky until the next capture; the context is not poisoned.
 */
gc_status gc_graph_status(gc_graph graph, void* stream);

/*
 * Test hook for the whole-step schedule, taken by every later gc_graph_capture
 * on `ctx` until changed: with fail_round >= 0 the combined-pass items of that
 * step wait for one more finished reorganisation part than the step has, so
 * their waits give up after fail_spins probes (0: the default bound, about a
 * second); fail_round < 0 turns the hook off.  Other waits keep their bound.
 * Every wave still ends normally and reads only buffers of its step; the
 * launch reports through gc_graph_status, and that step's accelerations are
 * unspecified.
 */
gc_status gc_debug_step_waits(gc_ctx ctx, uint32_t fail_spins, int32_t fail_round);

/* ---------------------------------------------------------------- tuning and introspection */

/*
 * Time the combined pass of a reorganised gravity batch for each candidate
 * and return the fastest in *best (other prm fields are copied from `base`).
 * Synchronises `stream`.  Two stages: the launch shape -- tiles {128, 256,
 * 512} x waves {2, 4, 8} x schedules {0, 1} x targets_per_lane {1, 2}, in
 * that nesting order, with every task in one launch -- then, with the best
 * shape, the aggregation count (Sec. 3.1: the number of requests combined
 * into one kernel): all tasks, twice, once and half the occupancy-sized
 * count (resident workgroups per CU x CUs).  times_ms (optional, 40 floats)
 * receives the average per candidate in that order (36 shapes, then 4
 * counts).
 * Tuning cache: with cache_path != NULL the result is kept in a JSON file
 * keyed by device (gfx name and CU count), force kind and a hash of the
 * batch's shape (tasks, targets, direct entries, node references and the
 * histogram of tasks by target count).  A key found there is returned
 * without timing (*from_cache = 1, times_ms untouched); otherwise the
 * candidates are timed and the entry is added (the file is rewritten whole,
 * other keys kept).  A file that is not such a cache gives GC_E_INVAL and is
 * left alone.  from_cache may be NULL.
 */
gc_status gc_autotune(gc_batch batch, const gc_force_params* base, const float* nodes_dev, float* acc_dev,
                      int32_t reps, float* times_ms, gc_force_params* best, const char* cache_path,
                      int32_t* from_cache, void* stream);

/*
 * In-cutoff pairs of a reorganised Lennard-Jones batch (Sec. 4.2: the pairs
 * of a patch pair within the cutoff carry the force work): pairs with
 * r^2 < r_cut^2 by the forward pass's FP32 decision, i < j in self tasks,
 * each pair of a task counted once.  The measure of algorithmic work against
 * which a pass's candidate evaluations are set.  Needs a device-resident
 * source; synchronises `stream`.
 */
gc_status gc_lj_count_pairs(gc_batch batch, float r_cut, int64_t* pairs, void* stream);

/* Occupancy of the combined gravity kernel: resident blocks per CU and CU count. */
gc_status gc_occupancy(gc_ctx ctx, const gc_force_params* prm, int32_t* blocks_per_cu, int32_t* n_cu);

/* ---------------------------------------------------------------- Ewald correction */

/*
 * Periodic gravity (Sec. 4.1: ChaNGa's Ewald summation kernel, combined like
 * the force requests, Sec. 4.3).  For a cubic box of side L holding total
 * mass M with centre of mass com, the correction at a target x, with
 * r = x - com taken to the nearest image, is the pull of every periodic image
 * of M plus the neutralising background, less the central copy's direct pull
 * (which the tree walk computes):
 *   a = G M [ sum_{n != 0} -(erfc(alpha s)/s^3 + 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec
 *           + (erf(alpha s)/s^3 - 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec   (n = 0)
 *           - 2/L^2 sum_h e^{-pi^2 |h|^2/(alpha L)^2}/|h|^2 sin(2 pi h.r/L) h ],
 * s_vec = r + n L over images n in {-nrep..nrep}^3 and wave vectors h in Z^3
 * with 0 < |h|^2 <= hmax2.  alpha = 0 takes 2 / L.
 *
 * S (xx, yy, zz, xy, xz, yz) is the box's second moment about com,
 * sum_j m_j (x_j - com)(x_j - com)^T; all zeros (the default) gives the
 * monopole alone.  Otherwise the same kernel psi~ (a = G M grad psi~ above)
 * is expanded to second order about com: a += G/2 S_ab grad d_a d_b psi~,
 * which per real-space image s_vec adds
 *   G [ 1/2 (tr(S) s_vec + 2 S s_vec) B_2(s) - 1/2 (s_vec.S.s_vec) s_vec B_3(s) ],
 *   B_l = ((2l - 1) B_{l-1} + (2 alpha^2)^l / (alpha sqrt(pi)) e^{-alpha^2 s^2}) / s^2,
 *   B_0 = erfc(alpha s)/s for n != 0 and -erf(alpha s)/s for n = 0 (there from
 *   its series below alpha s = 1),
 * and per wave vector
 *   G 4 pi^2 / L^4 e^{-pi^2 |h|^2/(alpha L)^2}/|h|^2 (h.S.h) sin(2 pi h.r/L) h.
 * Valid: L > 0, alpha >= 0, 0 <= nrep <= 4, 0 <= hmax2 <= 64, S finite
 * (GC_E_INVAL otherwise).
 */
typedef struct {
  float L, G, M;
  float com[3];
  float alpha;
  int32_t nrep;
  int32_t hmax2;
  float S[6];
} gc_ewald_params;

/*
 * Adds the correction to acc_dev (float4 [n_ids]; x, y, z) for every target of
 * every task of a reorganised gravity batch, in one launch, reading the
 * targets' records as the combined pass does.  Asynchronous.
 */
gc_status gc_launch_ewald(gc_batch batch, const gc_ewald_params* prm, float* acc_dev, void* stream);

/* ---------------------------------------------------------------- CPU/GPU scheduling */

/*
 * Dynamic scheduling of work requests between the CPU and the GPU (Sec. 3.3).
 * A request's workload is the number of input data items it reads.  After
 * each execution on a device the caller records its items and seconds; each
 * device keeps the running mean of its seconds per item.  gc_hybrid_split
 * gives the CPU the share tau_gpu / (tau_cpu + tau_gpu) of a queue's items:
 * scanning the queue from the front with a running sum of items, the prefix
 * up to the request at which the sum reaches that share goes to the CPU
 * (*n_cpu requests, *items_cpu items), the rest to the GPU; a share of zero
 * items gives the CPU nothing.  Until both devices have a record the share is
 * one half.  Pure host logic; GC_E_INVAL on bad arguments, state unchanged.
 */
enum { GC_DEVICE_CPU = 0, GC_DEVICE_GPU = 1 };
typedef struct gc_hybrid_* gc_hybrid;
gc_status gc_hybrid_create(gc_hybrid* out);
gc_status gc_hybrid_destroy(gc_hybrid h);
gc_status gc_hybrid_record(gc_hybrid h, int32_t device, int64_t items, double seconds);  /* items >= 1 */
gc_status gc_hybrid_split(gc_hybrid h, const int64_t* items, int32_t n, int32_t* n_cpu, int64_t* items_cpu);
gc_status gc_hybrid_state(gc_hybrid h, double* tau_cpu, double* tau_gpu, int64_t* runs_cpu, int64_t* runs_gpu);

/*
 * The CPU's Lennard-Jones kernel for the requests scheduled there: the same
 * force law, FP32 cutoff decision and force factor as the device pass (pair
 * sums in FP64), both atoms of every pair updated; acc += F / m (host float4
 * [n_ids], x y z; the caller zeroes it).  tasks / j_ranges as for
 * gc_submit_tasks (one j range per task), rec: host float4 [n_ids] records by
 * id; eps_t, sig_t, mass_t: host arrays of n_types.  n_threads: 0 = the
 * hardware's thread count (at most 64).  Synchronous; GC_E_INVAL on ranges
 * outside [0, n_ids), a type outside [0, n_types) or bad arguments (acc
 * unchanged), GC_E_NOMEM if the per-thread sums cannot be allocated.
 */
gc_status gc_lj_forces_cpu(const gc_task* tasks, int32_t n_tasks, const int32_t* j_ranges, int32_t n_ranges,
                           const float* rec, int32_t n_ids, int32_t n_types, const float* eps_t, const float* sig_t,
                           const float* mass_t, float r_cut, float* acc, int32_t n_threads);

/* ---------------------------------------------------------------- combining policy */

/*
 * When to launch a combined kernel over a stream of arriving work requests
 * (Sec. 3.1).  max_size is the number of requests that fill the GPU at full
 * occupancy; with one workgroup per request (GC_SCHED_TASKS) it is the
 * resident blocks per CU times the CU count (gc_occupancy).  The combiner
 * records the arrival times and keeps the largest interval seen between two
 * consecutive arrivals, max_interval.  At each poll: if at least max_size
 * requests wait, the first max_size of them are to be combined; otherwise, if
 * some wait and the time since the last arrival exceeds 2 * max_interval, all
 * of them are.  Requests leave in arrival order; the caller keeps them and
 * submits the ones taken into a batch.  Pure host logic: times are the
 * caller's clock in seconds, non-decreasing across arrive and poll calls
 * (GC_E_INVAL otherwise, state unchanged).  Before a second arrival no interval
 * is known (max_interval = 0), so a poll after any time has passed takes what
 * waits.  A combiner is not thread-safe.
 */
typedef struct gc_combiner_* gc_combiner;
gc_status gc_combiner_create(int32_t max_size, gc_combiner* out);  /* max_size >= 1 */
gc_status gc_combiner_destroy(gc_combiner comb);
/* n >= 1 requests arrive at time t (as n arrivals at the same instant: interval 0 between them). */
gc_status gc_combiner_arrive(gc_combiner comb, double t, int64_t n);
/* At time t: *take = the number of waiting requests to combine now (0: keep waiting); they leave
 * the waiting count.  *reason (may be NULL): 0 none, 1 max_size reached, 2 idle for 2 * max_interval. */
gc_status gc_combiner_poll(gc_combiner comb, double t, int64_t* take, int32_t* reason);
/* Waiting requests, max_interval (s), and the launches decided so far by each rule (any may be NULL). */
gc_status gc_combiner_state(gc_combiner comb, int64_t* waiting, double* max_interval, int64_t* n_full,
                            int64_t* n_idle);

#ifdef __cplusplus
}
#endif

#endif /* GCHARM_H */
