// Internal declarations shared by the kernels and the C-ABI host code of
// the gfx950 bisection-update library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cbtk {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kRankGrid = 2048;   // persistent workgroups of the per-bisector kernels (8 per CU)
constexpr int kWordsPerBlock = 1024;  // bitfield words per workgroup (enumeration)
constexpr int kReduceSub = 10;    // tree levels reduced inside one workgroup

// Command word of a live bisector, rewritten every frame (the pipeline's
// per-bisector command integer of Section 3.3, plus bookkeeping bits).
enum : uint32_t {
    kDecMask = 3u,
    kKeep = 0u,
    kSplit = 1u,
    kMerge = 2u,
    kMCfg = 1u << 2,   // member of a merge configuration (Alg. 4)
    kMQuad = 1u << 3,  // the configuration is a cycle of four (else a border pair)
    kMMin = 1u << 4,   // smallest heap ID of its configuration
    kMAcc = 1u << 5,   // merge reservation accepted (on the smallest member)
    kMUnan = 1u << 6,  // every member of the configuration decided MERGE
    kMExec = 1u << 7,  // configuration merges this frame (on every member)
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
    kStCount
};

struct Counters {
    uint32_t L;     // live blocks at frame start (CBT root)
    uint32_t F;     // free blocks
    uint32_t Tm;    // total merge reservation (saturated)
    uint32_t Ts;    // total split reservation (saturated)
    uint32_t N;     // allocations of this frame
    uint32_t err;   // sticky error flags
    uint32_t pad[2];
    uint32_t stat[kStCount];
};

// Device state of one instance, carved from the caller's workspace.
struct Pool {
    uint64_t* id;      // [cap] heap ID per block (stale when free)
    int4* link;        // [cap] twin, next, prev (block indices, -1 = border), unused
    uint32_t* cmd;     // [cap] command word, rewritten every frame
    uint4* fwd;        // [cap] per-frame forwarding / merge members
    float4* vflat;     // [3 cap] flat-domain vertices (xyz, w unused)
    float4* vworld;    // [3 cap] their world positions; w of the first holds
                       //         the subdivision depth, of the second the
                       //         parity of the heap ID (as integers)
    uint32_t* bits;    // [W]   occupancy bitfield, bit s&31 of word s>>5
    uint32_t* tree;    // [2^(D-4)] sum-reduction tree down to word level
    uint32_t* live;    // [cap] rank -> block, ascending
    uint32_t* freel;   // [cap] first N free blocks of the pre-frame bitfield
    uint32_t* list;    // [cap] per-workgroup compacted work lists (blocks), each
                       //       workgroup's entries from its first rank on: merge
                       //       candidates, then accepted initiators, then owners
    uint32_t* lcnt;    // [kRankGrid] entries in each workgroup's list
    uint2* part;       // [kRankGrid] per-workgroup partial sums
    Counters* ctr;
    float* root;       // [9H] root triangle vertices
    int32_t D, k, H;
    uint32_t cap, W;
};

// Per-frame LOD constants (Section 3.3 kernel 4), passed by value.
struct LodK {
    float cam[3], right[3], up[3], fwd[3];
    float f2, t2s, t2m, tx, ty, znear;
    const float* table;
    int32_t res;
    float amp;
    int32_t mode;
};

size_t workspace_layout(int32_t H, int32_t D, Pool* P, char* base);

// Optional event pair recorded around the launches of one pipeline stage
// (stage numbers of include/cbt.h).
struct StageEvents {
    int stage;
    hipEvent_t begin;
    hipEvent_t end;
};

hipError_t launch_frame(const Pool& P, const LodK& K, const uint8_t* decisions, hipStream_t s,
                        const StageEvents* ev);
hipError_t launch_reduce(const Pool& P, hipStream_t s);
hipError_t launch_enumerate(const Pool& P, hipStream_t s);
// rebuild the vertex cache of every live block (flat != 0: decode the flat
// vertices from the heap IDs first; otherwise recompute world positions)
hipError_t launch_refresh(const Pool& P, const LodK& K, int flat, hipStream_t s);
hipError_t launch_bits_from_ids(const Pool& P, hipStream_t s);
hipError_t launch_gather_ids(const Pool& P, uint32_t r0, uint32_t n, uint64_t* out, hipStream_t s);
hipError_t launch_gather_links(const Pool& P, uint32_t r0, uint32_t n, int32_t* out3, hipStream_t s);
hipError_t launch_gather_vertices(const Pool& P, uint32_t r0, uint32_t n, float* out9, hipStream_t s);
hipError_t launch_gather_decisions(const Pool& P, uint32_t L, uint8_t* out_per_slot, hipStream_t s);
hipError_t launch_export_heap(const Pool& P, uint32_t* out, hipStream_t s);

}  // namespace cbtk

