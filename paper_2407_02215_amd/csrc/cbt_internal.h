// Internal declarations shared by the kernels and the C-ABI host code of
// the gfx950 bisection-update library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cbtk {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kMaxRankGroups = 2048;   // rank workgroups of one instance, at most
constexpr int kMinRankGroups = 16;
constexpr int kWordsPerBlock = 256;    // bitfield words per workgroup (enumeration, free list)
constexpr int kMaxReduceSub = 10;      // tree levels reduced inside one workgroup, at most
constexpr int kMinReduceSub = 5;
constexpr int kMaxBatch = 4096;        // instances in one batched launch
constexpr uint32_t kMapShift = 20;     // block map entry: instance << 20 | local block

// Command word of a live bisector, rewritten every frame (the pipeline's
// per-bisector command integer of Section 3.3, plus bookkeeping bits).
enum : uint32_t {
    kDecMask = 3u,
    kKeep = 0u,
    kSplit = 1u,
    kMerge = 2u,
    kMCfg = 1u << 2,   // smallest member of a merge configuration (Alg. 4)
    kMQuad = 1u << 3,  // the configuration is a cycle of four (else a border pair)
    kMMin = 1u << 4,   // smallest heap ID of its configuration
    kMAcc = 1u << 5,   // merge reservation accepted (on the smallest member)
    kMUnan = 1u << 6,  // every member of the configuration decided MERGE
    kMExec = 1u << 7,  // configuration merges this frame
    kMarkB = 1u << 8,  // split marks: base edge, Next edge, Prev edge
    kMarkN = 1u << 9,
    kMarkP = 1u << 10,
    kMarks = 7u << 8,
    kDepthShift = 16,
    kDepthMask = 63u << 16,
};

// Sticky device-side error flags.
enum : uint32_t {
    kErrChain = 1u,      // compatibility chain did not end
    kErrPointer = 2u,    // neighbour pointer out of range / not mutual
    kErrAlloc = 4u,      // allocation beyond the free blocks
    kErrDecision = 8u,   // injected decision code > 2
    kErrEdge = 16u,      // edge pieces do not match across a shared edge
    kErrSpin = 32u,      // a persistent frame's wait for an earlier phase gave up
};

enum StatIndex {
    kStSplitReq = 0,
    kStMergeReq,
    kStMergeCfg,
    kStMergeAcc,
    kStSplitAcc,
    kStMergeExec,
    kStSplitConsumed,
    kStFrees,
    kStMergeCand,   // even members listed for the merge vote
    kStCount
};

// Workgroups add their frame statistics into one of kStLanes copies (one
// 128-byte line each, picked by workgroup index), not all into one word:
// device-wide atomics on one address serialise, and a thousand workgroups
// finishing together queued for tens of microseconds per pass.  The
// reduction's last kernel folds the copies into Counters::stat and clears
// them.
constexpr int kStLanes = 64;
constexpr int kLaneWords = 32;
static_assert(kStCount <= kLaneWords, "statistics of one lane in one line");

struct Counters {
    uint32_t L;     // live blocks at frame start (CBT root)
    uint32_t F;     // free blocks
    uint32_t N;     // allocations of this frame
    uint32_t err;   // sticky error flags
    uint32_t pad[2];
    uint32_t stat[kStCount];
};

// Per-frame LOD constants (Section 3.3 kernel 4), evaluated in double on
// the host.  Binary32 instances use each value rounded once to float,
// binary64 instances use it as is.
struct LodK {
    double cam[3], right[3], up[3], fwd[3];
    double f2, t2s, t2m, tx, ty, znear;   // t2s, t2m: squared pixel lengths, or twice the pixel areas
    double amp;
    const float* table;
    int32_t res;
    int32_t mode;
    int32_t crit;                          // size criterion (CBT_CRIT_*)
};

// The pointer record and the forwarding record of one block share a
// 32-byte line: a pass that finds a neighbour consumed reads its forwarding
// without another random access, and the fill writes a consumed bisector's
// fate and forwarding in one line.
struct LinkFwd {
    int4 l;    // twin, next, prev (blocks, -1 on a border) and the bisector's
               // fate this frame: 0 between frames; once the fill has run,
               // the command word of a bisector consumed by a split (marks
               // and depth), or kMExec for a merged member
    uint4 f;   // during a frame: blocks given to a split bisector's outputs,
               // or the parent block of a merged member; on the smallest
               // member of a merge configuration first its other members,
               // then (parent, members)
};

// Device state of one instance, carved from its workspace.
struct Pool {
    uint64_t* id;      // [cap] heap IDs as the last initialisation or import
                       //       wrote them; a frame keeps a block's ID in its
                       //       vertex record only
    LinkFwd* lf;       // [cap] pointer and forwarding records, side by side
    float4* vworld;    // [3 cap] world positions of the three vertices; the w
                       //         components hold raw bits: the subdivision depth
                       //         (first vertex), the heap ID's low and high words
                       //         (second and third); binary64 instances: [3 cap]
                       //         double4 with the depth and the whole heap ID
    uint32_t* cmd;     // [cap] command word, rewritten every frame
    uint32_t* bits;    // [W]   occupancy bitfield, bit s&31 of word s>>5 (one
                       //       word, partly used, when D < 5)
    uint32_t* tree;    // [2^(LW+1)] sum-reduction tree down to the word level
                       //       LW = word_level(D); node 1 is the root
    uint32_t* live;    // [cap] rank -> block, ascending
    uint32_t* freel;   // [cap] first N free blocks of the pre-frame bitfield
    uint2* list;       // [cap] per-workgroup compacted work lists, each
                       //       workgroup's entries from its first rank on:
                       //       merge candidates, then accepted initiators,
                       //       then owners with their command words
    uint32_t* lpre;    // [cap] beside each owner entry: outputs of the
                       //       workgroup's earlier owners
    uint32_t* lcnt;   // [kMaxRankGroups] entries in each workgroup's list
    uint2* part;       // [kMaxRankGroups] per-workgroup partial sums
    Counters* ctr;
    uint32_t* slane;   // [kStLanes][kLaneWords] frame statistics being summed
    float* root;       // [9H] root triangle vertices (binary64 instances: double)
    int32_t D, k, H;
    uint32_t cap, W;
    uint32_t G;        // rank workgroups (launch schedule)
    int32_t sub;       // tree levels per reduction workgroup (launch schedule)
    int32_t f64;       // vertices, world positions and the size test in binary64
};

// One instance as the kernels see it: state, this frame's constants and the
// injected decisions (NULL: LOD test).
struct Inst {
    Pool P;
    LodK K;
    const uint8_t* inj;
};

// Instances updated by the same launches.  Each block map holds, per
// workgroup of the batched grid, (instance << kMapShift) | workgroup within
// that instance's own grid.
struct Batch {
    int n;
    const Inst* inst;
    const uint32_t* map_rank;
    const uint32_t* map_word;
    const uint32_t* map_red;
    const uint32_t* map_list;
};

// Phases of one frame, in pipeline order (the persistent batched frame
// numbers its work items phase by phase).
enum Phase { kPhEnum = 0, kPhClass, kPhVote, kPhBudget, kPhWalk, kPhOwners, kPhFree, kPhFill, kPhResolve, kPhRedSub,
             kPhRedTop, kPhCount };

// Work list of a persistent batched frame: items [first[p], first[p+1])
// are phase p's items of every instance, instance by instance; an item is a
// span of consecutive workgroups of the instance's grid for the phase
// (persist_items_host); ticket hands the items out, done[i * kPhCount + p]
// counts instance i's finished items of phase p.  Both are cleared before
// each launch.
struct Persist {
    uint32_t* ticket;
    uint32_t* done;
    const uint32_t* map;   // per item: instance << kMapShift | span index
    uint32_t first[kPhCount + 1];
    uint32_t fail_phase;   // test hook: this stage's waits give up at once (kPhCount: none)
};

// Everything a launch sequence needs: either one instance passed by value
// (batched = false) or a batch in device memory, and the grid sizes.
struct Launch {
    bool batched;
    bool f64;          // every instance of the launch in binary64
    Inst one;
    Batch B;
    uint32_t n_inst;
    uint32_t grid_rank, grid_word, grid_red, grid_list;
    bool persistent;           // batched: one persistent launch per frame
    Persist W;
    uint32_t persist_groups;   // workgroups of that launch
};

// Tree level of the bitfield words: D - 5 (32 blocks per word), and 0 for a
// pool of fewer than 32 blocks, whose single partial word is the root.
__host__ __device__ inline int word_level(int D) { return D > 5 ? D - 5 : 0; }

// per-instance grid sizes
uint32_t word_groups(const Pool& P);
// workgroups of the passes over the compacted work lists (and of the LOD
// pass, two rank chunks each): half the rank workgroups rounded up, at
// least 16.  Their loads are dependent and random; fewer waves in flight
// measured faster than the rank passes' count
__host__ __device__ inline uint32_t list_groups(const Pool& P)
{
    const uint32_t h = (P.G + 1) / 2;
    return h > 16u ? h : 16u;
}
uint32_t reduce_groups(const Pool& P);
int reduce_levels(const Pool& P);

size_t workspace_layout(int32_t H, int32_t D, int32_t f64, Pool* P, char* base);
Launch single_launch(const Pool& P, const LodK& K, const uint8_t* inj);

// Optional event pair recorded around the launches of one pipeline stage
// (stage numbers of include/cbt.h).
struct StageEvents {
    int stage;
    hipEvent_t begin;
    hipEvent_t end;
};

hipError_t launch_frame(const Launch& X, hipStream_t s, const StageEvents* ev);
// workgroups of the persistent frame kernel that fit on the device at once (0
// on error)
uint32_t persist_resident_groups(bool f64);
// workgroups of instance P's grid in phase ph, and the persistent frame's
// items for them
uint32_t phase_groups_host(const Pool& P, int ph);
uint32_t persist_items_host(uint32_t groups);
hipError_t launch_reduce(const Launch& X, hipStream_t s);
hipError_t launch_enumerate(const Launch& X, hipStream_t s);
// rebuild the vertex cache of every live block: world positions (with the
// instance's K) of the vertices decoded from its heap ID
// from_ids: the heap IDs come from the ID array (after an initialisation or
// an import), else from the live blocks' own vertex records
hipError_t launch_refresh(const Launch& X, hipStream_t s, bool from_ids);

// cached world positions of the L live bisectors in rank order (after an
// enumeration) -> out9[9 L]
hipError_t launch_export_triangles(const Pool& P, uint32_t L, float* out9, hipStream_t s);

// the counters of every instance of a batch -> out[n_inst]
hipError_t launch_gather_counters(const Launch& X, Counters* out, hipStream_t s);

// single-instance helpers for queries, snapshot and restore
// IDs, pointer and forwarding records, commands, partials, counters -> cleared
hipError_t launch_clear_pool(const Pool& P, hipStream_t s);
// list lengths, partial sums and statistics lanes -> zero (frame scratch
// shared with other instances)
hipError_t launch_clear_frame_scratch(const Pool& P, hipStream_t s);
hipError_t launch_bits_from_ids(const Pool& P, hipStream_t s);
hipError_t launch_gather_ids(const Pool& P, uint32_t r0, uint32_t n, uint64_t* out, hipStream_t s);
hipError_t launch_gather_links(const Pool& P, uint32_t r0, uint32_t n, int32_t* out3, hipStream_t s);
// root halfedge and subdivision code (1 followed by the path bits) of ranks
// [r0, r0 + n); either output may be NULL
hipError_t launch_gather_canonical(const Pool& P, uint32_t r0, uint32_t n, int32_t* root_h, uint64_t* code,
                                   hipStream_t s);
hipError_t launch_gather_vertices(const Pool& P, uint32_t r0, uint32_t n, float* out9, hipStream_t s);
// binary64 decode (binary32 instances: their decode, widened)
hipError_t launch_gather_vertices64(const Pool& P, uint32_t r0, uint32_t n, double* out9, hipStream_t s);
hipError_t launch_gather_decisions(const Pool& P, uint32_t L, uint8_t* out_per_slot, hipStream_t s);
hipError_t launch_export_heap(const Pool& P, uint32_t* out, hipStream_t s);
// live bisectors in rank order (after an enumeration) <-> packed records
// (block, id low, id high, twin, next, prev); the import scatters into a
// cleared pool and flags blocks or pointers out of range
// into_cache: out6 lies in the pool's own vertex cache (the IDs are first
// copied to the ID array, so no record is overwritten before it is read)
hipError_t launch_export_live(const Pool& P, uint32_t L, uint32_t* out6, hipStream_t s, bool into_cache);
hipError_t launch_import_live(const Pool& P, uint32_t n, const uint32_t* in6, hipStream_t s);
// blocks [b0, b0+n) <-> packed records (id low, id high, twin, next, prev)
hipError_t launch_export_records(const Pool& P, uint32_t b0, uint32_t n, uint32_t* out5, hipStream_t s);
hipError_t launch_import_records(const Pool& P, uint32_t b0, uint32_t n, const uint32_t* in5, hipStream_t s);

}  // namespace cbtk
