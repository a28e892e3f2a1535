/*
 * cbt.h -- C ABI of the MI355X (gfx950) adaptive bisection update.
 *
 * Implements the per-frame update of "Concurrent Binary Trees for Large-Scale
 * Game Components" (Benyoub & Dupuy, 2024): root bisectors are the halfedges
 * of a polygon mesh (Section 2.2), every frame each live bisector is refined,
 * decimated or kept (Section 2.3, Alg. 3-6, Table 1), and the bisectors live
 * in a fixed pool of 2^D blocks managed by a concurrent binary tree -- a
 * bitfield with a sum-reduction tree -- used as a memory pool (Section 3.2,
 * Alg. 7-9) through the nine-step pipeline of Section 3.3.
 *
 * Conventions shared by every call
 *  - Status: every function returns cbt_status; 0 is CBT_OK, errors are
 *    negative.  No C++ exception crosses this boundary.  cbt_last_error()
 *    gives a message for the last failure on a handle.
 *  - Memory: the caller owns every array passed in.  Host arrays may be
 *    released when the call returns.  The device workspace given to cbt_init
 *    is owned by the caller (for instance a torch tensor), must hold
 *    cbt_workspace_bytes(H, D) bytes, be 256-byte aligned, and outlive the
 *    handle; the library allocates no device memory of its own.
 *  - Streams: the hipStream_t given to cbt_init is borrowed; every device
 *    operation of the handle is enqueued on it.  cbt_update and
 *    cbt_update_with_decisions do not synchronise unless statistics are
 *    requested; the query calls synchronise the stream.
 *  - Threads: a handle is not thread-safe; use one handle per thread or lock.
 *  - Heap IDs: root halfedge h is bisector 2^k + h with k = ceil(log2 H);
 *    the children of bisector x are 2x and 2x+1 (Section 2.3 "Notation",
 *    Section 3.3 "Initialization").  A bisector of depth d therefore has
 *    2^(k+d) <= x < 2^(k+d+1); 64-bit IDs allow d <= 63 - k.
 *  - Neighbour pointers are pool slots (-1 = border): twin across the edge
 *    (v0,v1), next across (v1,v2), prev across (v2,v0) of the vertex triple.
 */
#ifndef CBT_H
#define CBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cbt_status;
#define CBT_OK 0
#define CBT_E_ARG (-1)      /* null or out-of-range argument                 */
#define CBT_E_MESH (-2)     /* mesh fails validation (see cbt_init)           */
#define CBT_E_DEPTH (-3)    /* D < ceil(log2 H) or D > 30                     */
#define CBT_E_CAPACITY (-4) /* output arrays too small                        */
#define CBT_E_DEVICE (-5)   /* HIP error or device-side check; handle failed  */
#define CBT_E_BUDGET (-6)   /* workspace smaller than cbt_workspace_bytes     */
#define CBT_E_STATE (-7)    /* handle failed earlier                          */

typedef struct cbt_instance* cbt_handle;

/* Halfedge mesh (Section 2.1).  Host arrays of length H: Twin (-1 on a
 * border), Next, Prev and Vert (origin vertex) of every halfedge; pos holds
 * V vertices as x,y,z floats.  Requirements checked by cbt_init: H >= 3,
 * Next and Prev inverse permutations, every face cycle of length >= 3, Twin
 * an involution without fixed points whose halfedges run in opposite
 * directions and do not belong to the same corner (twin(h) is neither
 * next(h) nor prev(h)), vertex indices in [0, V). */
typedef struct {
    int32_t H;
    const int32_t* twin;
    const int32_t* next;
    const int32_t* prev;
    const int32_t* vert;
    int32_t V;
    const float* pos;
} cbt_mesh;

/* Pinhole camera: position, forward direction, up direction (need not be
 * orthogonal to forward), vertical field of view in radians, viewport in
 * pixels and near-plane distance along the forward axis. */
typedef struct {
    float pos[3];
    float fwd[3];
    float up[3];
    float fovy;
    int32_t width;
    int32_t height;
    float znear;
} cbt_camera;

/* World position applied to the flat-domain vertices before the LOD test
 * (Section 4.1: planets project vertices on a sphere and displace them;
 * terrains displace by an elevation map). */
enum {
    CBT_MODE_FLAT = 0,        /* p = v                                            */
    CBT_MODE_SPHERE = 1,      /* p = n (1 + amplitude T_cube(n)), n = v / |v|      */
    CBT_MODE_HEIGHTFIELD = 2  /* p = v + (0, 0, amplitude T_grid(v.x, v.y))        */
};

/* Size criteria of the screen-space test (the paper's size target of
 * Section 3.3 kernel 4 and Section 4.1). */
enum {
    CBT_CRIT_EDGE = 0,     /* projected length of the base edge, thresholds in pixels      */
    CBT_CRIT_AREA = 1,     /* projected area of the triangle, thresholds in pixels^2        */
    CBT_CRIT_DISTANCE = 2  /* base edge over its midpoint's distance, in pixels; cull-free  */
};

/* LOD parameters.  With CBT_CRIT_EDGE a live bisector is split when the
 * projected length of its base edge (v0,v1) exceeds split_px pixels and
 * merged when it is below merge_px, and one whose base edge reaches behind
 * the near plane is split; with CBT_CRIT_AREA the projected area of its
 * triangle is compared with split_px and merge_px (pixels^2), and one with
 * any vertex behind the near plane is split.  Either way one whose vertices
 * all lie outside one frustum plane is merged.  CBT_CRIT_DISTANCE is the
 * cull-free, distance-only variant: the base edge's length e and its
 * midpoint's distance r from the camera give f e / r pixels (f the focal
 * length in pixels) whatever the view direction, no frustum or near-plane
 * test, thresholds in pixels as for CBT_CRIT_EDGE.  The comparisons are
 * strict and division-free.
 * table is a DEVICE pointer (float32), caller-owned, that must stay valid
 * while updates run: 6 * table_res^2 texels for CBT_MODE_SPHERE (faces
 * +x,-x,+y,-y,+z,-z; texel (i,j) of a face at row j, column i) or
 * table_res^2 for CBT_MODE_HEIGHTFIELD (texel (i,j) at x = i/(res-1),
 * y = j/(res-1)); sampled bilinearly.  NULL for CBT_MODE_FLAT. */
typedef struct {
    int32_t mode;
    float split_px;
    float merge_px;
    const float* table;
    int32_t table_res;
    float amplitude;
    int32_t criterion;   /* CBT_CRIT_EDGE, CBT_CRIT_AREA or CBT_CRIT_DISTANCE */
} cbt_lod_params;

/* Per-frame counters (filled when a non-NULL pointer is passed). */
typedef struct {
    int64_t live_before;      /* L, the CBT root before the frame            */
    int64_t free_before;      /* F = 2^D - L                                  */
    int64_t split_requests;   /* bisectors whose decision is SPLIT            */
    int64_t split_accepted;   /* split initiators within the memory budget    */
    int64_t merge_requests;   /* bisectors whose decision is MERGE            */
    int64_t merge_configs;    /* unanimous merge configurations               */
    int64_t merge_accepted;   /* configurations within the memory budget      */
    int64_t merges_executed;  /* configurations merged                        */
    int64_t split_consumed;   /* bisectors consumed by splits                 */
    int64_t allocations;      /* new blocks                                   */
    int64_t frees;            /* released blocks                              */
    int64_t live_after;
    int64_t max_depth;        /* 0 unless requested through cbt_query         */
    int64_t merge_candidates; /* even MERGE members examined by the vote      */
} cbt_frame_stats;

/* Live bisectors in ascending slot order (two-call pattern: with capacity
 * smaller than the live count, only count is written and CBT_E_CAPACITY is
 * returned).  Every array pointer is a HOST pointer and may be NULL.
 * root_h / subdiv_id give each bisector in the paper's notation b_j^d
 * (Section 2.3 "Notation"): the root halfedge h it descends from and its
 * subdivision code, a leading 1 followed by its d path bits (most
 * significant first, 0 = first child): heap ID x of depth d has
 * h = (x >> d) - 2^k and subdiv_id = 2^d + (x mod 2^d).  The triangulation's
 * canonical form is the set of these pairs, which does not depend on the
 * pool slots (sort them to compare two triangulations). */
typedef struct {
    int64_t capacity;     /* in: entries available in the per-bisector arrays */
    int64_t count;        /* out: number of live bisectors                    */
    int32_t* slot;        /* out: pool slot                                   */
    uint64_t* heap_id;    /* out: heap ID                                     */
    int32_t* twin;        /* out: neighbour slots, -1 on a border             */
    int32_t* next;
    int32_t* prev;
    float* vertices;      /* out: 9 floats per bisector, flat-domain (Alg. 2)  */
    uint32_t* tree;       /* out: full CBT heap of 2^(D+1) counters, node 0 = 0 */
    double* vertices64;   /* out: 9 doubles per bisector, flat-domain (Alg. 2),
                             the binary64 decode of CBT_INIT_FP64 instances
                             (binary32 instances: their decode, widened)   */
    int32_t* root_h;      /* out: root halfedge of each bisector              */
    uint64_t* subdiv_id;  /* out: 1 followed by the bisector's path bits      */
} cbt_bisectors;

/* Device workspace needed for a mesh of H halfedges and a pool of 2^D
 * blocks (0 when the arguments are invalid). */
size_t cbt_workspace_bytes(int32_t H, int32_t D);

/* Section 3.3 "Initialization": H root bisectors in the first H blocks,
 * their neighbours copied from the halfedge operators, the first H bits
 * set, then the sum reduction.  Validates the mesh (CBT_E_MESH), requires
 * ceil(log2 H) <= D <= 30 (CBT_E_DEPTH; Section 3.3 "Memory
 * Requirements": the pool must hold every root bisector; a pool of fewer
 * than 32 blocks keeps one partial bitfield word whose count is the tree
 * root) and a large enough workspace (CBT_E_BUDGET).  Synchronises the
 * stream before returning. */
cbt_status cbt_init(const cbt_mesh* mesh, int32_t D, void* device_workspace,
                    size_t workspace_bytes, void* hip_stream, cbt_handle* out);

/* Instance flags of cbt_init_ex. */
#define CBT_INIT_FP64 1u   /* vertices, world positions and the size test in
                              binary64 (the paper evaluates planet vertices in
                              double precision, Section 4.2): root triangles
                              with the face mean in binary64, a 96-byte vertex
                              record per block, the frame constants unrounded */

/* Workspace of cbt_init_ex (0 when the arguments or flags are invalid). */
size_t cbt_workspace_bytes_ex(int32_t H, int32_t D, uint32_t flags);

/* cbt_init with instance flags (0 is cbt_init).  Unknown flags are
 * CBT_E_ARG.  The pool logic is the same at either precision; only the
 * decode, the world positions and the size test change width.  Binary64
 * instances export triangles rounded once to float. */
cbt_status cbt_init_ex(const cbt_mesh* mesh, int32_t D, uint32_t flags, void* device_workspace,
                       size_t workspace_bytes, void* hip_stream, cbt_handle* out);

/* One frame of the Section 3.3 pipeline: every live bisector decides by the
 * LOD test, splits propagate along compatibility chains (Alg. 3), merges
 * need all members of a configuration (Alg. 4), blocks are reserved against
 * the free count and allocated through the free bits of the CBT, neighbour
 * pointers are rewritten (Alg. 5, Alg. 6, Table 1), the bitfield and the
 * sum-reduction tree are updated.  Asynchronous on the handle's stream
 * unless stats is non-NULL (then it synchronises and also reports device
 * checks as CBT_E_DEVICE). */
cbt_status cbt_update(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod,
                      cbt_frame_stats* stats);

/* Test hook: the same frame with the LOD test replaced by one decision per
 * pool slot (0 keep, 1 split, 2 merge), read from a DEVICE array of 2^D
 * bytes.  Roots still never merge and no split passes the index width. */
cbt_status cbt_update_with_decisions(cbt_handle h, const uint8_t* device_decisions,
                                     cbt_frame_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * frame as cbt_update, with the same result, but the frame's scratch arrays
 * (rank list, free list, work lists, owner offsets, list lengths, partial
 * sums, statistics lanes) are taken from a static device array of
 * cbt_noalloc_scratch_bytes() bytes (about 20 MiB, one copy per GPU, held
 * until the process ends) instead of the handle's workspace.  The handle's
 * workspace still holds the state (IDs, pointer records, vertex cache,
 * commands, bitfield, tree, counters).  Limits and errors: pools of depth
 * D <= 20 only (CBT_E_CAPACITY beyond); the handle's device must be current
 * (CBT_E_ARG otherwise).  Allocates nothing: no hipMalloc, hipFree or event
 * creation; the static array's address is looked up once per device on the
 * first call.  Every call on one GPU shares that GPU's array: calls whose
 * work overlaps on the device (different streams, or different host threads
 * without ordering) race and corrupt each other's frames; serialise them on
 * one stream.  The array keeps the last call's contents; the accumulators
 * that must start at zero are cleared on the stream by each call.  After
 * it, cbt_query_decisions reports CBT_E_STATE (the rank list it needs is in
 * the shared array).  Asynchronous unless stats is non-NULL, as cbt_update. */
cbt_status cbt_update_noalloc(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod,
                              cbt_frame_stats* stats);
size_t cbt_noalloc_scratch_bytes(void);

/* Multi-pass mode: the update repeated with the same camera until a pass
 * changes nothing (no allocation, no release) or max_passes passes ran, for
 * cold starts and camera cuts (the single pass per frame of Section 3.3
 * refines at most one level per frame).  passes receives the passes run;
 * last, if non-NULL, the last pass's counters.  Synchronises after every
 * pass. */
cbt_status cbt_update_converge(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod,
                               int32_t max_passes, int32_t* passes, cbt_frame_stats* last);

/* Triangle export, the step after the update (Section 4.1: the leaves are
 * rasterised): the world positions of the three vertices (v0, v1, v2) of
 * every live bisector, in ascending block order, 9 floats per triangle,
 * written to the DEVICE array device_out of capacity triangles.  Shared
 * edges have bit-identical endpoints (watertight).  count receives the live
 * count; CBT_E_CAPACITY (nothing written) when it exceeds capacity.
 * Synchronises once (to read the count); the export itself is
 * asynchronous on the handle's stream. */
cbt_status cbt_export_triangles(cbt_handle h, float* device_out, int64_t capacity, int64_t* count);

/* Copies the live bisectors (and optionally vertices and the CBT heap) to
 * host arrays; synchronises the stream. */
cbt_status cbt_query(cbt_handle h, cbt_bisectors* out);

/* Decision codes of the last frame per slot (host array of 2^D bytes):
 * 0 keep, 1 split, 2 merge for slots live when the frame started, 255 for
 * the others.  Valid until the next update or query. */
cbt_status cbt_query_decisions(cbt_handle h, uint8_t* per_slot);

/* Snapshot / restore of the pool state as host arrays of 2^D entries
 * (heap ID 0 marks a free block).  Restore rebuilds the bitfield and the
 * sum-reduction tree from the IDs; the caller guarantees the arrays
 * describe a conforming triangulation of this mesh (for instance a snapshot
 * of the same instance).  Both synchronise the stream. */
cbt_status cbt_snapshot(cbt_handle h, uint64_t* heap_id, int32_t* twin, int32_t* next,
                        int32_t* prev);
cbt_status cbt_restore(cbt_handle h, const uint64_t* heap_id, const int32_t* twin,
                       const int32_t* next, const int32_t* prev);

/* Compact state transfer: the live bisectors only, in rank order, as 6
 * uint32 each (block, heap ID low, heap ID high, twin, next, prev), 24 bytes
 * per live bisector instead of a 2^D-entry snapshot.  cbt_export_live
 * writes them to the DEVICE array records of capacity entries (count
 * receives the live count; CBT_E_CAPACITY, nothing written, when it
 * exceeds capacity); it synchronises once to read the count, the copy
 * itself is asynchronous on the handle's stream.  cbt_import_live replaces
 * the handle's state by count records (a DEVICE array, or a HOST array when
 * on_host is non-zero) exported from an instance of the same mesh and
 * depth: the pool is cleared, the records scattered to their blocks, the
 * bitfield, the sum-reduction tree and the vertex cache rebuilt.  A block
 * or pointer out of range is reported as CBT_E_DEVICE (the handle is then
 * failed).  Synchronises the stream. */
cbt_status cbt_export_live(cbt_handle h, uint32_t* records, int64_t capacity, int64_t* count);
cbt_status cbt_import_live(cbt_handle h, const uint32_t* records, int64_t count, int32_t on_host);

/* LOD constants the device uses for a camera, evaluated once per frame in
 * double precision and rounded to float: cam[3] right[3] up[3] fwd[3] f^2
 * split_px^2 merge_px^2 tan_x tan_y znear (18 floats). */
cbt_status cbt_frame_constants(cbt_handle h, const cbt_camera* camera,
                               const cbt_lod_params* lod, float* out18);

/* Stage timing with HIP events on the handle's stream.  After
 * cbt_time_stage(h, stage), every later update records an event pair around
 * that stage's launches (at most 8192 pairs are kept; stage 0 disables and
 * clears).  cbt_stage_time synchronises and returns the number of timed
 * launches and their summed duration in milliseconds. */
enum {
    CBT_STAGE_NONE = 0,
    CBT_STAGE_ENUMERATE = 1,  /* frame set-up, live blocks in rank order       */
    CBT_STAGE_CLASSIFY = 2,   /* LOD test on the vertex cache, command words   */
    CBT_STAGE_VOTE = 3,       /* merge configurations, unanimity, reservations */
    CBT_STAGE_BUDGET = 4,     /* rank-order reservation cut                    */
    CBT_STAGE_CHAIN = 5,      /* compatibility-chain split marks               */
    CBT_STAGE_OWNERS = 6,     /* outputs per owner                             */
    CBT_STAGE_OFFSETS = 7,    /* no launch: the allocation offsets are scanned
                                 inside the free-list, fill and pointer passes */
    CBT_STAGE_FREELIST = 8,   /* free blocks                                   */
    CBT_STAGE_FILL = 9,       /* new heap IDs, forwarding records              */
    CBT_STAGE_RESOLVE = 10,   /* neighbour pointers, bitfield clears           */
    CBT_STAGE_REDUCE = 11,    /* sum-reduction tree                            */
    CBT_STAGE_FRAME = 12,     /* the whole update                              */
    CBT_STAGE_EXPORT = 13     /* cbt_export_triangles' kernel                  */
};
cbt_status cbt_time_stage(cbt_handle h, int32_t stage);
cbt_status cbt_stage_time(cbt_handle h, int64_t* launches, double* total_ms);
/* The same launches one by one (milliseconds each, in update order); count
 * receives their number, CBT_E_CAPACITY when capacity is smaller. */
cbt_status cbt_stage_times(cbt_handle h, double* out_ms, int64_t capacity, int64_t* count);

/* Launch schedule of the handle's per-bisector kernels (not part of the
 * method; results do not depend on it): rank_groups workgroups, each owning
 * a contiguous chunk of ceil(L / rank_groups) ranks, in [16, 2048], and
 * reduce_levels tree levels reduced inside one workgroup of the sum
 * reduction, in [5, 10].  The default is about one workgroup per 512 pool
 * blocks and 10 levels.  Takes effect at the next update. */
cbt_status cbt_set_schedule(cbt_handle h, int32_t rank_groups, int32_t reduce_levels);
cbt_status cbt_get_schedule(cbt_handle h, int32_t* rank_groups, int32_t* reduce_levels);

/* ---- Batched update ------------------------------------------------------
 * Many instances, of uneven mesh size and depth, advanced together: every
 * stage of the Section 3.3 pipeline is one launch whose workgroups are
 * spread over all member instances (each member keeps the schedule it had
 * when the batch was created), optionally captured once as a HIP graph and
 * replayed every frame.  Each member's result is the one cbt_update gives
 * (bit for bit): instances share launches, not state.
 *  - Memory: the caller owns a device workspace of
 *    cbt_batch_workspace_bytes(members, n) bytes (256-byte aligned) holding
 *    the instance descriptors, the counters and the block maps; the
 *    library allocates pinned host staging only.
 *  - Streams: all batch work runs on the batch's stream.  cbt_batch_create
 *    synchronises the members' own streams; afterwards the caller must not
 *    run work on a member concurrently with the batch.
 *  - Graphs: with CBT_BATCH_GRAPH (needs a non-null stream) the first
 *    update captures the kernel sequence; later updates upload the frame's
 *    descriptors (outside the graph) and replay it. */
typedef struct cbt_batch_s* cbt_batch;
#define CBT_BATCH_GRAPH 1
/* One persistent launch per frame instead of one launch per stage: the
 * resident workgroups take (stage, instance, workgroup) items in order from
 * a counter and each item waits until its instance has finished the
 * previous stage (per-instance counters), so instances proceed through the
 * pipeline independently (Section 3.3's nine kernels fused).  Same results
 * bit for bit.  A wait that exceeds its bound is reported as CBT_E_DEVICE
 * by the next update that reads statistics. */
#define CBT_BATCH_PERSISTENT 2

/* 0 when the member list is invalid (NULL, repeated or failed handles,
 * members of both precisions, n outside [1, 4096]). */
size_t cbt_batch_workspace_bytes(const cbt_handle* members, int32_t n);
cbt_status cbt_batch_create(const cbt_handle* members, int32_t n, void* device_workspace,
                            size_t workspace_bytes, void* hip_stream, int32_t flags,
                            cbt_batch* out);
/* One frame for every member: cameras[i], lods[i] as for cbt_update.  With
 * stats non-NULL (n entries) it synchronises and reports device checks as
 * CBT_E_DEVICE; otherwise it is asynchronous on the batch's stream. */
cbt_status cbt_batch_update(cbt_batch b, const cbt_camera* cameras, const cbt_lod_params* lods,
                            cbt_frame_stats* stats);
/* Test hook: device_decisions[i] as for cbt_update_with_decisions. */
cbt_status cbt_batch_update_with_decisions(cbt_batch b, const uint8_t* const* device_decisions,
                                           cbt_frame_stats* stats);
/* Releases the batch (not its workspace, not the members); synchronises. */
/* Test hook for the failure path of a persistent batch: every wait of the
 * given stage (1 .. 10: classify .. tree top, in pipeline order) gives up at
 * once, as a wait that ran out of its bound does; the instances' later
 * stages are skipped and the next update that reads statistics reports
 * CBT_E_DEVICE (the members are then failed).  -1 restores normal waits.
 * CBT_E_ARG for a batch that is not persistent.  Synchronises. */
cbt_status cbt_batch_fail_stage(cbt_batch b, int32_t stage);
cbt_status cbt_batch_destroy(cbt_batch b);

/* ---- Serving loop ----------------------------------------------------------
 * Tessellation-update requests (instance, camera) arrive at any time and are
 * batched continuously: whenever one of the server's launch slots is free,
 * every instance with a queued request and none in flight joins the next
 * batched frame (the cbt_batch path), which runs on that slot's own stream,
 * so batches overlap on the device.  At most one request per instance is in
 * flight and an instance's requests run in arrival order, so its states are
 * the ones cbt_update gives for the same cameras.
 *  - Memory: the caller owns one device arena (256-byte aligned).  Its first
 *    cbt_server_overhead_bytes(cfg) bytes hold the launch slots; instance
 *    workspaces (cbt_workspace_bytes each) are carved from the rest, up to
 *    memory_budget bytes.  An instance is admitted when its workspace fits;
 *    otherwise idle instances (none queued, none in flight) are evicted,
 *    least recently used first: their live records (cbt_export_live, 24
 *    bytes per live bisector) stay in the arena's top end and the workspace
 *    is released; when even the records do not fit, the oldest records move
 *    to host memory.  A request for an evicted instance re-admits it
 *    (cbt_init + cbt_import_live).  The server creates its own streams
 *    (default priority) and pinned host staging.
 *  - Latency of a request: from cbt_server_submit to the poll that observes
 *    its batch finished (host steady clock); queue_ms up to its launch.
 *  - Threads: a server is not thread-safe. */
typedef struct cbt_server_s* cbt_server;

typedef struct {
    int64_t memory_budget;  /* bytes for instance workspaces (0: the whole arena) */
    int32_t max_batch;      /* instances per batched launch, 1..4096            */
    int32_t slots;          /* batches in flight, each on its own stream, 1..8  */
    int64_t map_capacity;   /* workgroups per batched launch (all four grids)   */
} cbt_server_config;

typedef struct {
    uint64_t tag;           /* as given to cbt_server_submit                    */
    int64_t instance;
    int32_t status;         /* CBT_OK, or the reason the request failed         */
    int32_t batch_size;     /* instances in the batch that ran it               */
    double latency_ms;
    double queue_ms;
    int64_t live_before;
    int64_t live_after;
} cbt_completion;

typedef struct {
    int64_t instances, resident, queued, in_flight;
    int64_t requests, admissions, evictions, batches, frames;
    int64_t bisector_updates;   /* sum of live counts over served frames */
    int64_t bytes_resident, bytes_budget;   /* arena bytes in use (workspaces and records) */
    int64_t host_snapshots;                 /* evictions whose records went to host memory */
    double admit_ms, admit_ms_max;          /* host time spent admitting instances: total, longest */
    double evict_ms, evict_ms_max;          /* host time spent evicting instances: total, longest */
} cbt_server_stats;

size_t cbt_server_overhead_bytes(const cbt_server_config* cfg);   /* 0: invalid cfg */
cbt_status cbt_server_create(const cbt_server_config* cfg, void* device_arena, size_t arena_bytes,
                             cbt_server* out);
/* Registers an instance (the mesh is validated and copied; lod->table must
 * stay valid) and admits it if it fits; CBT_E_BUDGET if its workspace
 * exceeds the whole budget. */
cbt_status cbt_server_open(cbt_server s, const cbt_mesh* mesh, int32_t D, const cbt_lod_params* lod,
                           int64_t* instance_id);
cbt_status cbt_server_set_schedule(cbt_server s, int64_t instance_id, int32_t rank_groups,
                                   int32_t reduce_levels);
/* Launch schedules by (depth, live count) for the instances that have none
 * of their own (cbt_server_set_schedule): before each of an instance's
 * frames the server takes, among the n entries, those of the depth nearest
 * to the instance's (the deeper on a tie) and of them the one whose live
 * count is nearest by ratio to the instance's live count after its last
 * frame (its root count before the first).  Entries are checked as for
 * cbt_set_schedule (CBT_E_ARG); an entry whose grids exceed the block-map
 * capacity is skipped.  n = 0 clears the table.  Results do not depend on
 * schedules. */
cbt_status cbt_server_set_schedule_table(cbt_server s, int32_t n, const int32_t* depth, const int64_t* live,
                                         const int32_t* rank_groups, const int32_t* reduce_levels);
cbt_status cbt_server_submit(cbt_server s, int64_t instance_id, const cbt_camera* camera, uint64_t tag);
/* Collects finished batches, launches new ones, and returns up to capacity
 * completions (with wait != 0 it blocks until at least one batch ends when
 * none is ready). */
cbt_status cbt_server_poll(cbt_server s, int32_t wait, cbt_completion* out, int32_t capacity,
                           int32_t* count);
/* Runs until no request is queued or in flight (completions stay for poll). */
cbt_status cbt_server_drain(cbt_server s);
/* cbt_query of the instance's current state (waits for its request in
 * flight; re-admits it if evicted). */
cbt_status cbt_server_query(cbt_server s, int64_t instance_id, cbt_bisectors* out);
cbt_status cbt_server_close(cbt_server s, int64_t instance_id);
cbt_status cbt_server_get_stats(cbt_server s, cbt_server_stats* out);
cbt_status cbt_server_destroy(cbt_server s);

/* Number of live bisectors (synchronises). */
cbt_status cbt_live_count(cbt_handle h, int64_t* out);

/* Releases the handle (not the workspace).  Synchronises the stream. */
cbt_status cbt_destroy(cbt_handle h);

const char* cbt_status_string(cbt_status s);
const char* cbt_last_error(cbt_handle h);

#ifdef __cplusplus
}
#endif
#endif /* CBT_H */
