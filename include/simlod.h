/*
 * simlod.h -- C ABI of the MI355X octree LOD insertion library.
 *
 * The library keeps an octree level-of-detail structure resident in GPU
 * memory and inserts batches of points into it incrementally, following
 * "SimLOD: Simultaneous LOD Generation and Rendering" (Schuetz, Herzberger,
 * Wimmer, arXiv 2310.03567), section "Incrementally Updating the Octree":
 *
 *   1. expand: count the points reaching each leaf and split leaves that
 *      would exceed the leaf capacity, repeatedly, until none spills
 *      (subsection "Expanding the Octree");
 *   2. sample: project every point into the occupancy grid of each inner
 *      node on its path and create a voxel for every newly occupied cell
 *      (subsection "Voxel Sampling");
 *   3. allocate chunks for the new points and voxels and store them
 *      (subsections "Allocating Chunks" and "Storing Points and Voxels").
 *
 * Leaves hold the original points; inner nodes hold voxels sampled on an
 * R^3 grid (section "Octree"); both live in linked lists of fixed-size chunks
 * (section "Chunks and the Chunk Pool") carved out of one pre-allocated
 * persistent buffer (section "Persistent Buffer").
 *
 * Determinism.  A voxel takes the colour of the point with the smallest key
 * in its cell, key = position of the point in the cumulative insertion
 * sequence (the paper keeps the first point that reaches an empty cell; on a
 * GPU "first" is a race, so "first" is defined by key).  The resulting
 * octree is then a pure function of the cumulative point sequence,
 * independent of how it was cut into batches, and simlod_snapshot exports it
 * in a canonical order that a CPU implementation reproduces bit for bit.
 *
 * Threading and streams.  A handle must be used by one host thread at a
 * time.  Every call on a handle is enqueued on the stream passed to it; when
 * that is not the stream of the handle's previous call, the library first
 * makes it wait (with an event) for everything already enqueued on the
 * handle, so calls on one handle always run in call order.  Different
 * handles are independent.
 *
 * Errors.  Every function returns SIMLOD_OK (0) or a negative SIMLOD_ERR_*
 * code.  Capacity overflows detected on the device (node table, persistent
 * buffer, spill buffer, voxel backlog, work list) are recorded in a sticky
 * device status word and reported by a later call on the handle; the handle
 * is then POISONED: its octree is undefined, every call except
 * simlod_destroy, simlod_stats and simlod_status_string returns
 * SIMLOD_ERR_POISONED, and no kernel touches memory outside the library's
 * own buffers.
 */
#ifndef SIMLOD_H
#define SIMLOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIMLOD_ABI_VERSION 3

/* ---- status codes ---------------------------------------------------- */
#define SIMLOD_OK 0
#define SIMLOD_ERR_INVALID_ARGUMENT (-1) /* bad pointer, size or configuration   */
#define SIMLOD_ERR_OUT_OF_MEMORY (-2)    /* device or host allocation failed     */
#define SIMLOD_ERR_HIP (-3)              /* a HIP runtime call failed            */
#define SIMLOD_ERR_CAPACITY (-4)         /* a device-side capacity overflowed    */
#define SIMLOD_ERR_POISONED (-5)         /* handle unusable after an earlier error */
#define SIMLOD_ERR_KEY_SPACE (-6)        /* more than 2^32 - 1 points in one octree */
#define SIMLOD_ERR_NOT_FOUND (-7)        /* simlod_snapshot_subtree: no node with that path */
#define SIMLOD_ERR_BUSY (-8)             /* server: no stream slot or HBM budget free now */

/* Bits of simlod_stats_data.status_bits (device-side overflow causes). */
#define SIMLOD_OVF_NODES 0x1u   /* node table (max_nodes) full            */
#define SIMLOD_OVF_ARENA 0x2u   /* persistent buffer (arena_bytes) full    */
#define SIMLOD_OVF_SPILL 0x4u   /* spill buffer (spill_capacity) full      */
#define SIMLOD_OVF_BACKLOG 0x8u /* voxel backlog (backlog_capacity) full   */
#define SIMLOD_OVF_WORK 0x10u   /* expansion work list full                */
#define SIMLOD_OVF_HASH 0x20u   /* voxel claim table probe limit reached   */
#define SIMLOD_OVF_INTERNAL 0x40u /* internal consistency check failed     */
#define SIMLOD_OVF_HIST 0x80u   /* split histograms (hist_capacity) full    */

/* ---- records ---------------------------------------------------------- */

/* One point: XYZRGBA, 3 x float32 + 4 x uint8 = 16 bytes, the record format
 * the update consumes (section "Data Sets", SIM format).  Voxels use the
 * same record with xyz at the centre of their grid cell (section "Octree"). */
typedef struct simlod_point {
    float x, y, z;
    uint8_t r, g, b, a;
} simlod_point;

/* ---- configuration ----------------------------------------------------- */

/* Octree parameters and capacities.  Fill with simlod_default_config and
 * override what is needed.
 *
 * root_min, root_size  Cubic domain of the octree, fixed at creation (a
 *                      streamed cloud's final bounds are unknown).  Integer
 *                      coordinates: K = max_depth + grid_bits bits per axis,
 *                      scale = fl32(2^K / root_size),
 *                      q = clamp(floor(fl32(fl32(v - root_min) * scale)),
 *                      0, 2^K - 1), NaN -> 0.  Points outside the domain are
 *                      clamped for placement only; their records are stored
 *                      unchanged.
 * leaf_capacity        T: a leaf splits when it would hold more than T
 *                      points (section "Octree": 50,000).
 * grid_bits            r: inner nodes sample on an R^3 grid, R = 2^r
 *                      (section "Voxel Sampling Grid": 128^3, r = 7); 0..8.
 * max_depth            Dmax: depth of the deepest possible leaf (root = 0);
 *                      nodes at Dmax never split.  max_depth + grid_bits
 *                      must be <= 24, max_depth <= 21.
 * chunk_capacity       C: records per chunk (section "Chunks and the Chunk
 *                      Pool": 1000).  Changes layout only, never results.
 * max_nodes            Node table capacity (>= 9).
 * hist_capacity        Leaves that may be mid-split at once in one pass: each
 *                      takes a histogram of 4,680 counters (18.7 KB) of the
 *                      points below it, 4 levels deep; 0 = 8192.
 * arena_bytes          Persistent buffer for chunks, occupancy grids and
 *                      chunk tables; 0 = 90% of the free device memory left
 *                      after the other buffers (section "Persistent Buffer").
 * max_batch            Largest batch processed in one pass; larger inserts
 *                      are cut into consecutive passes of at most max_batch
 *                      points, which gives the identical octree.
 * spill_capacity       Points of split leaves re-inserted in one pass
 *                      (section "Expanding the Octree", spill buffer).
 * backlog_capacity     New voxels in one pass (section "Voxel Sampling"
 *                      suggests 10M).
 * device               HIP device ordinal.
 * arena_ptr            Caller-owned persistent buffer, or NULL (the library
 *                      allocates it).  Device memory of at least arena_bytes
 *                      (> 0) on `device`, 256-byte aligned, owned by the
 *                      caller (for instance a torch tensor), which must keep
 *                      it alive and untouched until simlod_destroy; the
 *                      library zeroes it at creation and never frees it.  The
 *                      paper's persistent buffer is one allocation made up
 *                      front (section "Persistent Buffer"); this lets the
 *                      caller's allocator make it.  Not accepted by the
 *                      server, which owns the memory of its octrees.
 */
typedef struct simlod_config {
    float root_min[3];
    float root_size;
    uint32_t leaf_capacity;
    uint32_t grid_bits;
    uint32_t max_depth;
    uint32_t chunk_capacity;
    uint32_t max_nodes;
    uint32_t hist_capacity;
    uint64_t arena_bytes;
    uint64_t max_batch;
    uint64_t spill_capacity;
    uint64_t backlog_capacity;
    int32_t device;
    uint32_t reserved1;
    void* arena_ptr;
} simlod_config;

/* Node record of the canonical export: preorder, children in octant order
 * 0..7 (octant bit 0 = x, bit 1 = y, bit 2 = z), all 8 children of an inner
 * node present.  path = 1 for the root, parent_path * 8 + octant below it.
 * count = points of a leaf or voxels of an inner node; the node's records
 * are records[first .. first + count), sorted by key.  24 bytes. */
typedef struct simlod_node_record {
    uint64_t path;
    uint64_t first;
    uint32_t count;
    uint8_t depth;
    uint8_t is_leaf;
    uint16_t reserved;
} simlod_node_record;

/* Canonical export buffers (two-call pattern, see simlod_snapshot). */
typedef struct simlod_snapshot_buffers {
    uint64_t num_nodes;         /* out */
    uint64_t num_records;       /* out: num_points + num_voxels */
    uint64_t num_points;        /* out */
    uint64_t num_voxels;        /* out */
    simlod_node_record* nodes;  /* in: host buffer of num_nodes, or NULL */
    simlod_point* records;      /* in: host buffer of num_records, or NULL */
    uint32_t* keys;             /* in: host buffer of num_records, or NULL; a
                                   leaf point's own key, or the key of the
                                   point that coloured a voxel */
} simlod_snapshot_buffers;

/* Counters of a handle (simlod_stats). */
typedef struct simlod_stats_data {
    uint64_t num_nodes, num_leaves, num_inner;
    uint64_t num_points, num_voxels;
    uint64_t chunks_in_use;      /* sum over nodes of ceil(count / C)          */
    uint64_t chunks_pooled;      /* freed chunks waiting for reuse             */
    uint64_t arena_bytes_used, arena_bytes_total;
    uint64_t batches;            /* insertion passes so far                    */
    uint64_t points_inserted;
    uint64_t last_rounds;        /* count/split rounds of the last pass        */
    uint64_t last_spilled;       /* points re-inserted from split leaves       */
    uint64_t last_new_voxels;    /* voxels created by the last pass            */
    uint64_t max_rounds, max_spilled, max_new_voxels; /* high-water marks     */
    uint64_t sum_rounds, sum_spilled, sum_new_voxels; /* totals over passes   */
    uint32_t status_bits;        /* SIMLOD_OVF_* bits, 0 when healthy          */
    int32_t poisoned;
} simlod_stats_data;

/* Per-kernel timing, recorded with HIP events around each launch when
 * enabled by simlod_set_kernel_timing.  Index = SIMLOD_KERNEL_*. */
#define SIMLOD_KERNEL_COUNT 0        /* expansion: first-round leaf counts */
#define SIMLOD_KERNEL_SPLIT 1        /* expansion: first-round split        */
#define SIMLOD_KERNEL_ALLOC_POINTS 2 /* expansion rounds 3..R (usually none) and
                                        chunk allocation for leaves: one launch */
#define SIMLOD_KERNEL_SAMPLE_STORE 3 /* voxel claims + point stores         */
#define SIMLOD_KERNEL_ALLOC_VOXELS 4 /* chunk allocation for inner nodes    */
#define SIMLOD_KERNEL_STORE_VOXELS 5 /* voxel stores                        */
#define SIMLOD_KERNEL_FINISH 6       /* group passes: status words for the
                                        host (the bookkeeping runs in the
                                        voxel store)                        */
#define SIMLOD_KERNEL_COUNT_HIST 7   /* expansion: split histograms         */
#define SIMLOD_KERNEL_BUILD 8        /* expansion: multi-level subtree build
                                        (round 2)                           */
#define SIMLOD_KERNEL_GROUP_BATCH 9  /* passes of one octree and 4M+ points:
                                        the batch grouped by spatial
                                        bucket                              */
#define SIMLOD_NUM_KERNELS 10
typedef struct simlod_kernel_times {
    uint64_t launches[SIMLOD_NUM_KERNELS];
    double total_ms[SIMLOD_NUM_KERNELS];
} simlod_kernel_times;

typedef struct simlod_octree simlod_octree; /* opaque handle */

/* ---- functions --------------------------------------------------------- */

/* Fills *cfg with the paper's parameters (T = 50,000, 128^3 grid, chunks of
 * 1,000, section "Octree") and default capacities: unit cube at the origin,
 * max_depth 16, 2^20 nodes, 8192 split histograms, arena 0 (= 90% of free
 * memory), max_batch 10M,
 * spill 16M, backlog 10M (section "Voxel Sampling"), device 0. */
int simlod_default_config(simlod_config* cfg);

/* Creates an empty octree (a single empty root leaf) on cfg->device.  All
 * device memory is allocated here, as the paper allocates its persistent
 * buffer once up front and carves nodes, chunks and grids out of it
 * (section "Persistent Buffer"; leaf capacity, grid size and chunk size from
 * section "Octree"); inserting device-resident points never allocates.
 * The handle owns its memory until simlod_destroy.  *out is written only on
 * success.  Errors: INVALID_ARGUMENT (NULL pointers,
 * parameters outside the ranges above), OUT_OF_MEMORY, HIP. */
int simlod_create(const simlod_config* cfg, simlod_octree** out);

/* Inserts n points (the next n keys of the cumulative sequence): one
 * update of section "Incrementally Updating the Octree" per max_batch points
 * (expand, voxel-sample, allocate and store; the paper inserts the batches
 * loaded for a frame one after another, section "Overview").
 * pts: device or host pointer to n simlod_point records (16-byte aligned for
 * device memory); host memory is copied to a library staging buffer first.
 * The points are borrowed until the stream work completes and never
 * retained.  stream: hipStream_t (NULL = the default stream); the call only
 * enqueues work and returns.  n = 0 is a no-op.
 * Errors: INVALID_ARGUMENT (NULL handle, NULL pts with n > 0), KEY_SPACE,
 * POISONED, CAPACITY (an earlier pass overflowed; handle now poisoned), HIP. */
int simlod_insert_batch(simlod_octree* h, const simlod_point* pts, uint64_t n, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * insertion as simlod_insert_batch, identical octree, but host input is
 * staged through a static device array of the library instead of a staging
 * buffer the library allocates, so the call never allocates or frees device
 * memory (the passes use only buffers allocated by simlod_create).
 * Limit: host input of at most 1,048,576 points per call (16 MiB array, one
 * per device, held until the process ends); larger host input returns
 * INVALID_ARGUMENT with simlod_last_error naming the limit.  Device input
 * needs no staging and has no such limit.  All calls on one device share
 * the array, which keeps the last call's points: calls that overlapped on a
 * device would race on it, so the library serializes them -- a host lock per
 * device around the staging, and on the device each call's copy into the
 * array waits (with an event) for the passes of the previous call that read
 * it, whatever handle, thread or stream made that call.
 * Errors: as simlod_insert_batch, plus INVALID_ARGUMENT for the limit. */
int simlod_insert_batch_static(simlod_octree* h, const simlod_point* pts, uint64_t n,
                               void* stream);

/* Canonical export of the whole octree: the intermediate result the paper
 * displays while points are still streaming in (section "Introduction").
 * Synchronizes the handle's last stream.  Call with all
 * three buffer pointers NULL to obtain the sizes, then with host buffers of
 * at least those sizes (the octree must not change in between).  With only
 * `nodes` set, fills the node records alone (no record copy).  The library
 * allocates temporary device memory here.
 * Errors: INVALID_ARGUMENT (records or keys NULL but not both, or set
 * without nodes), POISONED, CAPACITY, OUT_OF_MEMORY, HIP. */
int simlod_snapshot(simlod_octree* h, simlod_snapshot_buffers* s);

/* Canonical export of one subtree: the node with `path` (1 = root, then
 * parent * 8 + octant per level, the same paths the snapshot records carry)
 * and all its descendants, in the same form and with the same two-call
 * pattern as simlod_snapshot; paths and depths stay absolute, `first`
 * counts from the subtree's first record.  Reads part of a large octree
 * (the intermediate results the paper displays while loading, section
 * "Introduction") without copying all of it to the host.
 * Errors: as simlod_snapshot; INVALID_ARGUMENT for a value that is not a
 * path or is deeper than max_depth; NOT_FOUND when an ancestor of the node
 * is a leaf (the node does not exist yet). */
int simlod_snapshot_subtree(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s);

/* The export of one node alone: its node record (path, depth, leaf flag,
 * count; first = 0) and its records sorted by key, with the same two-call
 * pattern as simlod_snapshot; what a renderer streams for one visible node
 * (section "Introduction": intermediate results are displayed while
 * loading).  Errors: as simlod_snapshot_subtree. */
int simlod_snapshot_node(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s);

/* The same export read the way a renderer consumes the layout: one
 * workgroup per node starts at the node's first chunk and follows each
 * chunk's next link (section "Chunks and the Chunk Pool"; the paper's
 * listing reads a node's chunks this way), instead of the per-node chunk
 * tables simlod_snapshot_subtree uses.  Identical output; a chunk list that
 * ends early or continues past the node's last chunk returns HIP with
 * simlod_last_error naming it. */
int simlod_snapshot_linked(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s);

/* Counters; synchronizes the handle's last stream.  Works on a poisoned
 * handle (status_bits tells why). */
int simlod_stats(simlod_octree* h, simlod_stats_data* st);

/* Waits for all work enqueued on the handle; reports device-side errors. */
int simlod_sync(simlod_octree* h);

/* Empties the octree (single empty root, key sequence restarts at 0) and
 * keeps all allocations; clears a poisoned state.  Enqueued on stream. */
int simlod_reset(simlod_octree* h, void* stream);

/* Frees everything; safe on a poisoned handle; NULL is a no-op. */
int simlod_destroy(simlod_octree* h);

/* Selects the kernels whose launches later passes bracket with HIP events on
 * the pass's stream: bit k of kernel_mask = SIMLOD_KERNEL_k (0 disables,
 * 0x1FF times all).  Clears the accumulated times. */
int simlod_set_kernel_timing(simlod_octree* h, uint32_t kernel_mask);

/* Synchronizes and returns the times accumulated since timing was enabled. */
int simlod_get_kernel_times(simlod_octree* h, simlod_kernel_times* out);

/* ---------------------------------------------------------------------
 * Batched insertion: one pass over a group of octrees.
 *
 * A group inserts one batch into each of up to SIMLOD_MAX_GROUP octrees
 * (all on one device) with a single sequence of kernel launches whose work
 * is the members' batches together: small batches of many clouds fill the
 * GPU as one large batch does (the paper inserts one cloud's batches in
 * turn, section "Incrementally Updating the Octree").  Each member's octree
 * is exactly the one its own simlod_insert_batch calls would give.
 * --------------------------------------------------------------------- */
#define SIMLOD_MAX_GROUP 128

typedef struct simlod_group simlod_group;

#define SIMLOD_GROUP_GRAPH 0x1u    /* replay passes from one captured hipGraph */
#define SIMLOD_GROUP_AUTOTUNE 0x2u /* tune the launch shape on the first passes */

/* Creates a group over `count` distinct handles of one device (the handles
 * stay owned by the caller and must outlive the group; while the group is
 * in use a member must not be inserted into through another call at the
 * same time).  flags: SIMLOD_GROUP_*.
 * With SIMLOD_GROUP_AUTOTUNE the first SIMLOD_TUNE_PASSES passes try
 * candidate workgroup counts for the point-parallel kernels (timed with HIP
 * events, which synchronizes those passes), then keep the fastest per
 * kernel.  With SIMLOD_GROUP_GRAPH, once the shape is settled, the pass is
 * captured into a hipGraph on first use and later passes replay it with
 * only the first kernel's arguments changed.
 * Errors: INVALID_ARGUMENT (NULL, count 0 or > SIMLOD_MAX_GROUP, repeated
 * or poisoned handles, mixed devices), OUT_OF_MEMORY, HIP. */
int simlod_group_create(simlod_octree* const* members, uint32_t count, uint32_t flags,
                        simlod_group** out);

/* Inserts pts[i][0..n[i]) into member i for every i (n[i] may be 0).  Every
 * pts[i] with n[i] > 0 must be 16-byte-aligned device memory.  Members'
 * batches larger than their max_batch are cut into several passes.
 * Enqueued on `stream`; returns after enqueueing.
 * Errors: INVALID_ARGUMENT, KEY_SPACE (some member would pass 2^32 - 1
 * points; nothing is enqueued), POISONED (a member is), CAPACITY (a member
 * overflowed in an earlier group pass; it is now poisoned), HIP. */
int simlod_group_insert(simlod_group* g, const simlod_point* const* pts, const uint64_t* n,
                        void* stream);

#define SIMLOD_TUNE_PASSES 10

/* The launch shape in use: the largest workgroup count of the point
 * counting, histogram counting, sampling/store and voxel-store kernels, and
 * whether tuning has finished (1) and a graph is captured (bit 1). */
int simlod_group_shape(simlod_group* g, uint32_t caps[4], uint32_t* state);

/* Times passes of the group per kernel (as simlod_set_kernel_timing). */
int simlod_group_set_kernel_timing(simlod_group* g, uint32_t kernel_mask);
int simlod_group_get_kernel_times(simlod_group* g, simlod_kernel_times* out);

/* Waits for the group's passes; reports members' device-side errors. */
int simlod_group_sync(simlod_group* g);

/* Releases the group (not its members); NULL is a no-op. */
int simlod_group_destroy(simlod_group* g);

/* Chunk-capacity autotuner: inserts the sample (device memory, 16-byte
 * aligned) into a scratch octree built from *cfg with each candidate
 * chunk_capacity in turn, timing the passes with HIP events on `stream`,
 * and returns the fastest candidate in *best (and its time in *best_ms, if
 * not NULL).  The chunk size changes memory layout and speed, never the
 * canonical octree (section "Chunks and the Chunk Pool" measures the
 * trade-off).  Scratch octrees are created and destroyed one at a time.
 * Errors: as simlod_create and simlod_insert_batch. */
int simlod_tune_chunk_capacity(const simlod_config* cfg, const simlod_point* sample, uint64_t n,
                               const uint32_t* candidates, uint32_t count, void* stream,
                               uint32_t* best, double* best_ms);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of insertion requests.
 *
 * A server keeps the octrees of its open streams resident on one device and
 * runs a request loop on its own host threads.  Each pass takes the oldest
 * queued request of every stream that has one and inserts them together
 * (one group pass, see simlod_group_insert), so requests that arrive while
 * others are on the GPU join the next pass; up to two passes are in flight,
 * so the device does not idle while requests wait.  A stream's requests are
 * applied in submission order, so each octree is exactly what inserting its
 * requests alone, in order, gives (the paper streams batches of one cloud
 * into one octree, section "Incrementally Updating the Octree").
 * --------------------------------------------------------------------- */
typedef struct simlod_server simlod_server;

typedef struct simlod_server_config {
    int device;
    uint32_t max_streams;       /* open octrees at once, 1..SIMLOD_MAX_GROUP */
    uint64_t hbm_budget;        /* device bytes the open octrees may hold */
    uint32_t max_per_pass;      /* requests per pass (0 = one per stream);
                                   1 serves requests one at a time, in
                                   arrival order: the unbatched form */
    uint32_t pass_points;       /* time budget of a pass, in points: a request
                                   in device memory larger than this is
                                   inserted over several passes, pass_points
                                   at a time (the paper's per-frame budget
                                   with the rest resumed next frame, section
                                   "Evaluation"), so small requests of other
                                   streams need not wait for one large
                                   update; it completes with its last part.
                                   The octree is the same (consecutive
                                   passes of one sequence).  0 = no budget;
                                   requests in host memory are never cut. */
    uint64_t staging_bytes;     /* device staging for requests in host memory
                                   (allocated at create; 0 = host requests
                                   are rejected) */
} simlod_server_config;

int simlod_server_create(const simlod_server_config* cfg, simlod_server** out);

/* Device bytes simlod_create allocates for *cfg, a caller-owned arena_ptr
 * buffer not included (arena_bytes must be set:
 * a served octree cannot take "90% of free memory"). */
int simlod_config_device_bytes(const simlod_config* cfg, uint64_t* bytes);

/* Admits an octree with configuration *cfg (its device must be the
 * server's; arena_bytes set): reuses a pooled octree when one fits (see
 * simlod_server_close), else allocates one; BUSY when no stream slot is free
 * or its device bytes would exceed the budget even with the pool released;
 * *id names the stream. */
int simlod_server_open(simlod_server* sv, const simlod_config* cfg, uint32_t* id);

/* Queues the insertion of pts[0..n) into stream id; the caller keeps the
 * points valid until the request completes.  *ticket identifies the request.
 * Returns at once.  pts is 16-byte-aligned device memory, or host memory
 * when the server has staging_bytes: the server's uploader thread then
 * copies the request into the device staging area on a copy stream of its
 * own as soon as space is free, while earlier passes run (the paper's
 * uploader thread copies loaded batches to a GPU-side queue asynchronously,
 * section "Overview"); the pass that takes the request waits for its copy.
 * Pinned host memory makes the copy asynchronous; pageable memory is copied
 * through the runtime's own staging.  A request's latency includes its
 * upload.
 * Errors: INVALID_ARGUMENT (also: host memory without staging, or a request
 * larger than staging_bytes), KEY_SPACE, POISONED (the stream's octree is). */
int simlod_server_submit(simlod_server* sv, uint32_t id, const simlod_point* pts, uint64_t n,
                         uint64_t* ticket);

/* State of a request: *done = 1 once its pass has completed; *latency_ms
 * (may be NULL) = completion - submission, host clock.  Returns the
 * request's own status: CAPACITY if its stream overflowed. */
int simlod_server_poll(simlod_server* sv, uint64_t ticket, int* done, double* latency_ms);

/* Blocks until every request submitted so far has completed. */
int simlod_server_drain(simlod_server* sv);

/* The stream's octree handle, for snapshots and stats once its requests
 * have completed (owned by the server; NULL if id is not open). */
simlod_octree* simlod_server_octree(simlod_server* sv, uint32_t id);

/* Closes a stream and returns at once: no more submissions; once its
 * queued requests have completed its slot frees up and its octree joins the
 * server's pool.  Pooled octrees keep their device memory (and budget): a
 * later open reuses the smallest one whose buffers fit the new
 * configuration, reconfigured and reset on the server's stream, so a running
 * server neither allocates nor frees device memory (either synchronizes the
 * device and stalls the passes).  An open that fits no pooled octree and
 * exceeds the budget releases pooled octrees, largest first. */
int simlod_server_close(simlod_server* sv, uint32_t id);

/* Blocks until every closed stream's slot has been freed. */
int simlod_server_wait_closed(simlod_server* sv);

/* Counters: passes launched, requests completed, points inserted, device
 * bytes held by open octrees. */
int simlod_server_counters(simlod_server* sv, uint64_t out[4]);

/* Stops the loop, closes every stream; NULL is a no-op. */
int simlod_server_destroy(simlod_server* sv);

/* Static description of a status code. */
const char* simlod_status_string(int code);

/* Text naming the HIP call behind the calling thread's most recent
 * SIMLOD_ERR_HIP or SIMLOD_ERR_OUT_OF_MEMORY, or the path behind its most
 * recent SIMLOD_ERR_NOT_FOUND ("" if none); valid until the thread's next
 * library call. */
const char* simlod_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIMLOD_H */
