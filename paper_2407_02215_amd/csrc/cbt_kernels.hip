// gfx950 kernels of the per-frame adaptive bisection update.
//
// One frame (the nine-kernel pipeline of Section 3.3) runs as a fixed
// sequence of launches on one stream.  Every per-bisector launch is a
// persistent grid of G workgroups per instance, each owning a contiguous
// chunk of ranks, bounded by device-resident counts (HIP has no indirect
// dispatch).  Cheap passes over every rank (in rank order, with workgroup
// scans) alternate with heavy passes over compacted per-workgroup work
// lists, so divergent pointer work runs with full wavefronts:
//
//   enumerate  L = CBT root, F = 2^D - L (its first workgroup)       (kernel 1)
//              rank -> block list; each workgroup's base comes from the
//              tree (the prefix form of the Alg. 7 descent)          (kernel 2)
//   classify   LOD test on the cached world positions -> command word;
//              split reservations per workgroup; list: even members
//              that decided MERGE                                   (kernels 3-4)
//   vote       (list) merge configuration (Alg. 4), smallest member,
//              unanimity; merge reservations per workgroup           (kernel 4)
//   budget     rank-order cut: merges first, then splits of 3d+4 blocks,
//              against F; list: accepted initiators                  (kernel 4)
//   walk       (list) split marks along compatibility chains (Alg. 3
//              as a closure, atomicOr)                               (kernel 4)
//   owners     outputs per owner; list: owners and command words     (kernel 5)
//   freelist   the first N zero bits of the pre-frame bitfield
//              (ZeroToBitID order, Alg. 8), bits set                (kernels 5, 8)
//   fill       (list) allocation offsets, vertex-cache records of the
//              outputs, forwarding records of consumed bisectors     (kernel 6)
//   resolve    (list) heap IDs and pointers of every new bisector,
//              back-pointers of untouched neighbours (Table 1, Alg. 5,
//              Alg. 6 and compositions); consumed bits cleared      (kernels 7-8)
//   reduce     sum-reduction tree in LDS                             (kernel 9)
//
// Every kernel exists in two forms: one instance passed by value in the
// kernel arguments, or a batch of instances in device memory, where a block
// map sends each workgroup of the batched grid to its instance.
//
// Determinism: allocation by scans in rank order (no atomic counter), one
// writer per pointer field, the only atomics are order-free bitwise OR/AND
// and counter additions.
//
// Vertex cache: every block keeps the world positions of its bisector's
// vertices.  A split decodes the parent's flat-domain vertices from its heap
// ID (Alg. 2, a few ALU operations per level), copies the parent's cached
// world positions and evaluates only the new midpoints; merged parents copy
// their children's.  The cache equals the world positions of the decode bit
// for bit, and the LOD test reads it instead of decoding d levels and
// sampling the displacement table three times.
//
// Floating point: IEEE binary32, no contraction (-ffp-contract=off),
// correctly rounded division and square root.

#include "cbt_internal.h"

#pragma clang fp contract(off)

namespace cbtk {

// Ranks each thread of a rank-order pass loads before it processes them
// (all rows' loads in flight at once: these passes are bound by the latency
// of the rank -> block -> command chain, not by bandwidth).
constexpr int kClassRows = 4;   // LOD test: 48 bytes of vertices per rank
// Rank chunks per workgroup of the LOD pass, which runs on the rank grid:
// one chunk per workgroup (G workgroups) measured 71.6 us per terrain
// frame against 76.6 us for two chunks on half as many workgroups.
constexpr uint32_t kClassChunks = 1;
// The rank-order scans (budget, owners) give each thread kSeg consecutive
// ranks: one workgroup scan per kBlock * kSeg ranks, and the segment of
// rank-list entries is one 16-byte load (4 ranks measured 22 + 28 us per
// terrain frame for the two scans against 24 + 35 us with 8).  Rank chunks
// are whole segments.
constexpr int kSeg = 4;

// ---------------------------------------------------------------------------
// wave64 / workgroup scan primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b)
{
    uint32_t s = a + b;
    return (s < a || s > 0x7fffffffu) ? 0x7fffffffu : s;
}

__device__ __forceinline__ uint2 sat_add2(uint2 a, uint2 b)
{
    return make_uint2(sat_add(a.x, b.x), sat_add(a.y, b.y));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint2 wave_incl_scan_sat(uint2 v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t tx = __shfl_up(v.x, o, 64);
        uint32_t ty = __shfl_up(v.y, o, 64);
        if (lane >= o) v = sat_add2(v, make_uint2(tx, ty));
    }
    return v;
}

// exclusive scan over the kBlock threads of a workgroup; sh holds >= 4 words
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        uint32_t t = sh[i];
        pre += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// inclusive saturating scan of pairs; sh holds >= 4 uint2
__device__ __forceinline__ uint2 block_incl_scan_sat(uint2 v, uint2* sh, uint2* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint2 inc = wave_incl_scan_sat(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint2 pre = make_uint2(0, 0), tot = make_uint2(0, 0);
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        uint2 t = sh[i];
        if (i < w) pre = sat_add2(pre, t);
        tot = sat_add2(tot, t);
    }
    __syncthreads();
    *total = tot;
    return sat_add2(pre, inc);
}

// exclusive saturating scan of pairs; sh holds >= 4 uint2
__device__ __forceinline__ uint2 block_excl_scan_sat(uint2 v, uint2* sh, uint2* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint2 inc = wave_incl_scan_sat(v);
    if (lane == 63) sh[w] = inc;
    uint2 ex = make_uint2(__shfl_up(inc.x, 1, 64), __shfl_up(inc.y, 1, 64));
    if (lane == 0) ex = make_uint2(0, 0);
    __syncthreads();
    uint2 pre = make_uint2(0, 0), tot = make_uint2(0, 0);
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const uint2 t = sh[i];
        if (i < w) pre = sat_add2(pre, t);
        tot = sat_add2(tot, t);
    }
    __syncthreads();
    *total = tot;
    return sat_add2(pre, ex);
}

// saturating sum of pairs over the workgroup, returned to every thread;
// sh holds >= 4 uint2
__device__ __forceinline__ uint2 block_reduce_sat2(uint2 v, uint2* sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = sat_add2(v, make_uint2(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64)));
    if (lane == 0) sh[w] = v;
    __syncthreads();
    uint2 t = make_uint2(0, 0);
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t = sat_add2(t, sh[i]);
    __syncthreads();
    return t;
}

// exclusive scan of pairs (plain sums); sh holds >= 4 uint2
__device__ __forceinline__ uint2 block_excl_scan2(uint2 v, uint2* sh, uint2* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint2 inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t tx = __shfl_up(inc.x, o, 64), ty = __shfl_up(inc.y, o, 64);
        if (lane >= o) inc = make_uint2(inc.x + tx, inc.y + ty);
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint2 pre = make_uint2(0, 0), tot = make_uint2(0, 0);
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const uint2 t = sh[i];
        if (i < w) pre = make_uint2(pre.x + t.x, pre.y + t.y);
        tot = make_uint2(tot.x + t.x, tot.y + t.y);
    }
    __syncthreads();
    *total = tot;
    return make_uint2(pre.x + inc.x - v.x, pre.y + inc.y - v.y);
}

// set lanes of a wave mask below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* sh)
{
    uint32_t t;
    (void)block_excl_scan(v, sh, &t);
    return t;
}

// saturating sum over the workgroup, returned to every thread; sh holds >= 4
__device__ __forceinline__ uint32_t block_sum_sat(uint32_t v, uint32_t* sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = sat_add(v, __shfl_xor(v, o, 64));
    if (lane == 0) sh[w] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t = sat_add(t, sh[i]);
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// instance selection
// ---------------------------------------------------------------------------

// The instance a workgroup serves and the workgroup's index in that
// instance's own grid: from the kernel arguments, or through a block map.
template <bool kB>
__device__ __forceinline__ uint32_t pick(const Batch& B, const Inst& one, const uint32_t* map, Pool& P)
{
    if constexpr (kB) {
        const uint32_t e = map[blockIdx.x];
        P = B.inst[e >> kMapShift].P;
        return e & ((1u << kMapShift) - 1u);
    } else {
        P = one.P;
        return blockIdx.x;
    }
}

template <bool kB>
__device__ __forceinline__ uint32_t pick_k(const Batch& B, const Inst& one, const uint32_t* map, Pool& P, LodK& K,
                                           const uint8_t*& inj)
{
    if constexpr (kB) {
        const uint32_t e = map[blockIdx.x];
        const Inst& I = B.inst[e >> kMapShift];
        P = I.P;
        K = I.K;
        inj = I.inj;
        return e & ((1u << kMapShift) - 1u);
    } else {
        P = one.P;
        K = one.K;
        inj = one.inj;
        return blockIdx.x;
    }
}

// one workgroup per instance
template <bool kB>
__device__ __forceinline__ void pick_inst(const Batch& B, const Inst& one, Pool& P)
{
    if constexpr (kB) P = B.inst[blockIdx.x].P;
    else P = one.P;
}

// ranks per rank workgroup: ceil(L / G) rounded up to whole segments
__device__ __forceinline__ uint32_t rank_chunk(uint32_t L, uint32_t G)
{
    const uint32_t c = (L + G - 1) / G;
    return (c + kSeg - 1) / kSeg * kSeg;
}

// ranks of workgroup blk: a contiguous chunk
__device__ __forceinline__ void rank_range(uint32_t L, uint32_t G, uint32_t blk, uint32_t* r0, uint32_t* r1)
{
    const uint32_t chunk = rank_chunk(L, G);
    const uint64_t a = (uint64_t)blk * chunk;
    const uint64_t b = a + chunk;
    *r0 = (uint32_t)(a < L ? a : L);
    *r1 = (uint32_t)(b < L ? b : L);
}

// The lists of all rank workgroups form one list in rank order.  Consumers
// share it evenly: each workgroup scans the list lengths into LDS
// (base[w] = entries before workgroup w's, base[G] = total) and takes a
// contiguous 1/G of the entries, so the work no longer follows where in
// rank order the split and merge activity happens to be.
struct ListShare {
    uint32_t i0, i1;      // this workgroup's entries [i0, i1)
    uint32_t chunk;       // ranks per rank workgroup
};

// With obase non-NULL the owners' output counts (the partials the owner
// pass leaves) are scanned the same way: obase[w] = outputs of the rank
// workgroups before w, obase[G] = N.
__device__ __forceinline__ ListShare list_share(const Pool& P, uint32_t blk, uint32_t* base, uint32_t* sh,
                                                uint32_t* obase = nullptr, uint32_t GL = 0)
{
    constexpr int E = kMaxRankGroups / kBlock;
    const uint32_t G = P.G;
    uint32_t v[E], o[E], loc = 0, oloc = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t w = threadIdx.x * E + e;
        v[e] = w < G ? P.lcnt[w] : 0u;
        o[e] = (obase && w < G) ? P.part[w].x : 0u;
        loc += v[e];
        oloc += o[e];
    }
    uint32_t tot, otot = 0;
    uint32_t run = block_excl_scan(loc, sh, &tot);
    uint32_t orun = obase ? block_excl_scan(oloc, sh, &otot) : 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t w = threadIdx.x * E + e;
        if (w < G) {
            base[w] = run;
            if (obase) obase[w] = orun;
        }
        run += v[e];
        orun += o[e];
    }
    if (threadIdx.x == 0) {
        base[G] = tot;
        if (obase) obase[G] = otot;
    }
    __syncthreads();
    if (!GL) GL = list_groups(P);   // the workgroups sharing the list
    const uint32_t per = (tot + GL - 1) / GL;
    const uint64_t a = (uint64_t)blk * per, b = a + per;
    ListShare s;
    s.i0 = (uint32_t)(a < tot ? a : tot);
    s.i1 = (uint32_t)(b < tot ? b : tot);
    s.chunk = rank_chunk(P.ctr->L, G);
    return s;
}

// position in P.list of entry i of the concatenated list (base[0] <= i <
// base[G]); *w receives the rank workgroup that wrote it
__device__ __forceinline__ uint32_t list_at(const uint32_t* base, uint32_t G, uint32_t chunk, uint32_t i,
                                            uint32_t* w)
{
    uint32_t lo = 0, hi = G;   // base[lo] <= i < base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= i) lo = mid;
        else hi = mid;
    }
    *w = lo;
    return lo * chunk + (i - base[lo]);
}

// The same from a rank workgroup known not to lie after entry i's
// (base[*w] <= i): a thread's entries increase, so its last result is the
// next start, and the scan moves a step or two instead of a binary search.
__device__ __forceinline__ uint32_t list_at_from(const uint32_t* base, uint32_t chunk, uint32_t i, uint32_t* w)
{
    uint32_t v = *w;
    while (base[v + 1] <= i) ++v;
    *w = v;
    return v * chunk + (i - base[v]);
}

// the rank workgroup of this workgroup's first entry (0 for an empty share)
__device__ __forceinline__ uint32_t share_start(const uint32_t* base, uint32_t G, const ListShare& ls)
{
    uint32_t w = 0;
    if (ls.i0 < ls.i1) (void)list_at(base, G, ls.chunk, ls.i0, &w);
    return w;
}

// block numbers of ranks [t0, t0 + kSeg); t0 is a multiple of kSeg below
// the pool size, so the 16-byte loads stay inside the rank list; ranks
// from r1 on read as block 0 (in bounds, unused)
__device__ __forceinline__ void load_seg(const Pool& P, uint32_t t0, uint32_t r1, uint32_t (&s)[kSeg])
{
    static_assert(kSeg % 4 == 0, "whole 16-byte loads per segment");
    uint4 q[kSeg / 4];
#pragma unroll
    for (int i = 0; i < kSeg / 4; ++i) q[i] = make_uint4(0, 0, 0, 0);
    if (t0 < r1) {
        const uint4* p = reinterpret_cast<const uint4*>(P.live + t0);
#pragma unroll
        for (int i = 0; i < kSeg / 4; ++i) q[i] = p[i];
    }
#pragma unroll
    for (int i = 0; i < kSeg / 4; ++i) {
        const uint32_t v[4] = {q[i].x, q[i].y, q[i].z, q[i].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) s[4 * i + k] = t0 + 4 * i + k < r1 ? v[k] : 0u;
    }
}

__device__ __forceinline__ int ilog2_64(uint64_t x) { return 63 - __clzll((long long)x); }

__device__ __forceinline__ void raise_err(const Pool& P, uint32_t e) { atomicOr(&P.ctr->err, e); }

__device__ __forceinline__ bool slot_ok(const Pool& P, int32_t s) { return (uint32_t)s < P.cap; }

// a workgroup's contribution to frame statistic k (one lane per workgroup
// index modulo kStLanes)
__device__ __forceinline__ void stat_add(const Pool& P, uint32_t blk, int k, uint32_t v)
{
    if (v) atomicAdd(&P.slane[(blk % kStLanes) * kLaneWords + k], v);
}

__device__ __forceinline__ int depth_of_cmd(uint32_t c) { return (int)((c & kDepthMask) >> kDepthShift); }

// The blocks of a bitfield word that exist: all 32, or the first 2^D of the
// single word of a pool smaller than one word (D < 5).  Bits past the pool
// never count as live and are never handed out as free.
__device__ __forceinline__ uint32_t word_valid(const Pool& P)
{
    return P.cap >= 32u ? 0xffffffffu : ((1u << P.cap) - 1u);
}

// Number of set bits in the words before word w, read off the tree: the
// left siblings along w's path from the root.  Their indices follow from
// w's bits alone, so the lanes of the first wave load one level each, all
// at once, and sum them; the result reaches every thread of the workgroup
// through sh_out (one barrier, which every thread must reach).
__device__ uint32_t ones_before_word(const Pool& P, uint32_t w, uint32_t* sh_out)
{
    if (threadIdx.x < 64) {
        const int LW = word_level(P.D);   // LW <= 25 < 64
        const int l = (int)threadIdx.x;
        uint32_t v = 0;
        if (l < LW && ((w >> l) & 1u)) {
            const uint32_t node = (1u << (LW - 1 - l)) | (w >> (l + 1));   // the path's node above level l
            v = P.tree[2 * node];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (threadIdx.x == 0) *sh_out = v;
    }
    __syncthreads();
    return *sh_out;
}

// ---------------------------------------------------------------------------
// kernel: frame begin (one workgroup per instance)
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// kernel: frame set-up and enumeration of the live blocks (rank order =
// ascending block index).  Each 256-word step is staged in LDS so the rank
// list is written coalesced.
// ---------------------------------------------------------------------------

struct Lds_enumerate {
    uint32_t sh[8];
    uint32_t stage[kBlock * 32];
    uint32_t sb;
};

__device__ __forceinline__ void run_enumerate(const Pool& P, uint32_t blk, Lds_enumerate& S_)
{
    auto& sh = S_.sh;
    auto& stage = S_.stage;
    auto& sb = S_.sb;
    if (blk == 0) {
        // frame set-up (kernel 1): L = the CBT root, F = 2^D - L, counters
        // cleared; no other workgroup reads the counters
        if (threadIdx.x == 0) {
            const uint32_t L = P.tree[1];
            P.ctr->L = L;
            P.ctr->F = P.cap - L;
            P.ctr->N = 0;
        }
        if (threadIdx.x < kStCount) P.ctr->stat[threadIdx.x] = 0;
    }
    const uint32_t w0 = blk * kWordsPerBlock;
    if (w0 >= P.W) return;
    // all of this workgroup's words in flight while the tree is descended
    constexpr int kSteps = kWordsPerBlock / kBlock;
    uint32_t words[kSteps];
    const uint32_t valid = word_valid(P);
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
        const uint32_t w = w0 + j * kBlock + threadIdx.x;
        words[j] = (w < P.W) ? (P.bits[w] & valid) : 0u;
    }
    uint32_t base = ones_before_word(P, w0, &sb);
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
        const uint32_t it = j * kBlock;
        const uint32_t w = w0 + it + threadIdx.x;
        uint32_t word = words[j];
        uint32_t tot;
        uint32_t o = block_excl_scan(__popc(word), sh, &tot);
        while (word) {
            const int bit = __ffs(word) - 1;
            stage[o++] = w * 32u + (uint32_t)bit;
            word &= word - 1;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < tot; i += kBlock)
            if (base + i < P.cap) P.live[base + i] = stage[i];
        __syncthreads();
        base += tot;
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_enumerate(Batch B, Inst one)
{
    __shared__ Lds_enumerate S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_word, P);
    run_enumerate(P, blk, S_);
}

// ---------------------------------------------------------------------------
// bisector geometry (Eq. 1 / Alg. 2), world position and the LOD test
// ---------------------------------------------------------------------------

// Vertices, world positions and the size test are generic in the precision
// R: binary32, or binary64 for instances created with the binary64 flag (the
// paper's planets are evaluated in double, Section 4.2).  The binary32 path
// uses every frame constant rounded once to float.

template <typename R>
struct Vec3 {
    R x, y, z;
};
using V3 = Vec3<float>;

template <typename R> struct Store;
template <> struct Store<float> { using T4 = float4; };
template <> struct Store<double> { using T4 = double4; };
template <typename R> using T4 = typename Store<R>::T4;

__device__ __forceinline__ float floor_r(float x) { return floorf(x); }
__device__ __forceinline__ double floor_r(double x) { return floor(x); }
__device__ __forceinline__ float abs_r(float x) { return fabsf(x); }
__device__ __forceinline__ double abs_r(double x) { return fabs(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return __builtin_sqrt(x); }

// The w components of a vertex record carry the subdivision depth (first
// vertex) and the heap ID (binary32: low and high words in the second and
// third vertices; binary64: the whole ID in the second), as raw bits that
// are only ever moved, never computed with.
__device__ __forceinline__ float4 make4(Vec3<float> v, uint32_t w) { return make_float4(v.x, v.y, v.z, __uint_as_float(w)); }
__device__ __forceinline__ double4 make4(Vec3<double> v, uint64_t w)
{
    return make_double4(v.x, v.y, v.z, __longlong_as_double((long long)w));
}
__device__ __forceinline__ int w_int(float w) { return __float_as_int(w); }
__device__ __forceinline__ int w_int(double w) { return (int)__double_as_longlong(w); }

template <typename R> struct RecId;
template <> struct RecId<float> {
    static __device__ __forceinline__ uint64_t get(const float4& b, const float4& c)
    {
        return (uint64_t)__float_as_uint(b.w) | ((uint64_t)__float_as_uint(c.w) << 32);
    }
    static __device__ __forceinline__ uint32_t low(const float4& b) { return __float_as_uint(b.w); }
};
template <> struct RecId<double> {
    static __device__ __forceinline__ uint64_t get(const double4& b, const double4&)
    {
        return (uint64_t)__double_as_longlong(b.w);
    }
    static __device__ __forceinline__ uint32_t low(const double4& b) { return (uint32_t)__double_as_longlong(b.w); }
};

template <typename R>
__device__ __forceinline__ Vec3<R> ld3(const T4<R>& v) { return {v.x, v.y, v.z}; }

template <typename R>
__device__ __forceinline__ Vec3<R> mid3(Vec3<R> a, Vec3<R> b)
{
    const R h = (R)0.5;
    return {(a.x + b.x) * h, (a.y + b.y) * h, (a.z + b.z) * h};
}

template <typename R>
__device__ __forceinline__ T4<R>* world_rec(const Pool& P, uint32_t s)
{
    return reinterpret_cast<T4<R>*>(P.vworld) + 3 * (size_t)s;
}

// Heap ID of a live block, from its vertex record (the frame keeps it there
// only; the ID array holds the IDs of the last initialisation or import).
__device__ __forceinline__ uint64_t block_id(const Pool& P, uint32_t s)
{
    if (P.f64) {
        const double4* r = world_rec<double>(P, s);
        return RecId<double>::get(r[1], r[2]);
    }
    const float4* r = world_rec<float>(P, s);
    return RecId<float>::get(r[1], r[2]);
}

// Splitting matrices applied from the root downwards, one path bit per
// level, most significant first: M0 -> (v0, v2, m), M1 -> (v2, v1, m).
// Scalar registers only (struct selects would be lowered through scratch).
template <typename R>
__device__ __forceinline__ void decode(const Pool& P, uint64_t id, int d, Vec3<R>& A, Vec3<R>& B, Vec3<R>& C)
{
    const int64_t h = (int64_t)(id >> d) - ((int64_t)1 << P.k);
    const R* r = reinterpret_cast<const R*>(P.root) + 9 * h;
    R ax = r[0], ay = r[1], az = r[2];
    R bx = r[3], by = r[4], bz = r[5];
    R cx = r[6], cy = r[7], cz = r[8];
    const R half = (R)0.5;
    for (int i = d - 1; i >= 0; --i) {
        const bool bit = (id >> i) & 1u;
        const R mx = (ax + bx) * half, my = (ay + by) * half, mz = (az + bz) * half;
        const R nax = bit ? cx : ax, nay = bit ? cy : ay, naz = bit ? cz : az;
        const R nbx = bit ? bx : cx, nby = bit ? by : cy, nbz = bit ? bz : cz;
        ax = nax; ay = nay; az = naz;
        bx = nbx; by = nby; bz = nbz;
        cx = mx; cy = my; cz = mz;
    }
    A = {ax, ay, az};
    B = {bx, by, bz};
    C = {cx, cy, cz};
}

__device__ __forceinline__ bool valid_id(const Pool& P, uint64_t id)
{
    const int d = ilog2_64(id) - P.k;
    return id != 0 && d >= 0 && d <= 63 - P.k && (int64_t)(id >> d) - ((int64_t)1 << P.k) < P.H;
}

template <typename R>
__device__ __forceinline__ R bilinear(const float* T, int res, R s, R t)
{
    R fs = floor_r(s), ft = floor_r(t);
    const R lim = (R)(res - 2);
    fs = fs < (R)0 ? (R)0 : fs;
    fs = fs > lim ? lim : fs;
    ft = ft < (R)0 ? (R)0 : ft;
    ft = ft > lim ? lim : ft;
    int i0 = (int)fs, j0 = (int)ft;
    i0 = i0 < 0 ? 0 : (i0 > res - 2 ? res - 2 : i0);   // bounds guard (no-op unless NaN)
    j0 = j0 < 0 ? 0 : (j0 > res - 2 ? res - 2 : j0);
    const R fx = s - fs, fy = t - ft;
    const float* r0 = T + (size_t)j0 * res + i0;
    const float* r1 = r0 + res;
    const R a = r0[0], b = r0[1], c = r1[0], e = r1[1];
    const R top = a + fx * (b - a);
    const R bot = c + fx * (e - c);
    return top + fy * (bot - top);
}

// cube-map face = axis of largest magnitude (ties x, y, z), face order
// +x -x +y -y +z -z, (u, v) = the other two components over the major one
template <typename R>
__device__ __forceinline__ R sample_cube(const LodK& K, R x, R y, R z)
{
    const R ax = abs_r(x), ay = abs_r(y), az = abs_r(z);
    int f;
    R u, v;
    if (ax >= ay && ax >= az) {
        f = x >= (R)0 ? 0 : 1;
        u = y / ax;
        v = z / ax;
    } else if (ay >= az) {
        f = y >= (R)0 ? 2 : 3;
        u = x / ay;
        v = z / ay;
    } else {
        f = z >= (R)0 ? 4 : 5;
        u = x / az;
        v = y / az;
    }
    const R hr = (R)0.5 * (R)(K.res - 1);
    return bilinear<R>(K.table + (size_t)f * K.res * K.res, K.res, (u + (R)1) * hr, (v + (R)1) * hr);
}

// world position of a flat-domain point (sphere projection + cube-map
// displacement, or height-field displacement, or identity)
template <typename R>
__device__ __forceinline__ Vec3<R> world(const LodK& K, Vec3<R> v)
{
    if (K.mode == 1) {
        const R len = sqrt_r((v.x * v.x + v.y * v.y) + v.z * v.z);
        const R nx = v.x / len, ny = v.y / len, nz = v.z / len;
        const R h = sample_cube<R>(K, nx, ny, nz);
        const R sc = (R)1 + (R)K.amp * h;
        return {nx * sc, ny * sc, nz * sc};
    }
    if (K.mode == 2) {
        const R r1 = (R)(K.res - 1);
        const R h = bilinear<R>(K.table, K.res, v.x * r1, v.y * r1);
        return {v.x, v.y, v.z + (R)K.amp * h};
    }
    return v;
}

// Screen-space size test without division (projected base-edge length, or
// projected triangle area): returns the decision code from the three world
// positions.
template <typename R>
__device__ __forceinline__ uint32_t lod_decide(const LodK& K, Vec3<R> p0, Vec3<R> p1, Vec3<R> p2)
{
    const R cam[3] = {(R)K.cam[0], (R)K.cam[1], (R)K.cam[2]};
    if (K.crit == 2) {
        // cull-free, distance-only: the base edge seen face-on from its
        // midpoint's distance r, f |p1 - p0| / r pixels, compared squared;
        // no frustum test, whatever the view direction
        const R h = (R)0.5;
        const R qx = (p0.x + p1.x) * h - cam[0], qy = (p0.y + p1.y) * h - cam[1], qz = (p0.z + p1.z) * h - cam[2];
        const R r2 = (qx * qx + qy * qy) + qz * qz;
        const R ex = p1.x - p0.x, ey = p1.y - p0.y, ez = p1.z - p0.z;
        const R A = (R)K.f2 * ((ex * ex + ey * ey) + ez * ez);
        if (A > (R)K.t2s * r2) return kSplit;
        if (A < (R)K.t2m * r2) return kMerge;
        return kKeep;
    }
    const Vec3<R> p[3] = {p0, p1, p2};
    const R rt[3] = {(R)K.right[0], (R)K.right[1], (R)K.right[2]};
    const R up[3] = {(R)K.up[0], (R)K.up[1], (R)K.up[2]};
    const R fw[3] = {(R)K.fwd[0], (R)K.fwd[1], (R)K.fwd[2]};
    const R tx = (R)K.tx, ty = (R)K.ty, znear = (R)K.znear;
    R vx[3], vy[3], vz[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const R q0 = p[i].x - cam[0], q1 = p[i].y - cam[1], q2 = p[i].z - cam[2];
        vx[i] = (q0 * rt[0] + q1 * rt[1]) + q2 * rt[2];
        vy[i] = (q0 * up[0] + q1 * up[1]) + q2 * up[2];
        vz[i] = (q0 * fw[0] + q1 * fw[1]) + q2 * fw[2];
    }
    bool on = true, ol = true, orr = true, ob = true, ot = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const R zx = tx * vz[i], zy = ty * vz[i];
        on = on && (vz[i] < znear);
        orr = orr && (vx[i] > zx);
        ol = ol && (vx[i] < -zx);
        ot = ot && (vy[i] > zy);
        ob = ob && (vy[i] < -zy);
    }
    if (on || ol || orr || ob || ot) return kMerge;
    const R f2 = (R)K.f2, t2s = (R)K.t2s, t2m = (R)K.t2m;
    if (K.crit == 1) {
        // projected triangle area: twice the area in pixels^2 is
        // f^2 |N| / (z0^2 z1 z2), N the cross product of the projected edges
        // with the depths multiplied out
        if (vz[0] < znear || vz[1] < znear || vz[2] < znear) return kSplit;
        const R ax = vx[1] * vz[0] - vx[0] * vz[1];
        const R ay = vy[1] * vz[0] - vy[0] * vz[1];
        const R bx = vx[2] * vz[0] - vx[0] * vz[2];
        const R by = vy[2] * vz[0] - vy[0] * vz[2];
        const R N = ax * by - bx * ay;
        const R A = f2 * abs_r(N);
        const R zq = (vz[0] * vz[0]) * (vz[1] * vz[2]);
        if (A > t2s * zq) return kSplit;
        if (A < t2m * zq) return kMerge;
        return kKeep;
    }
    if (vz[0] < znear || vz[1] < znear) return kSplit;
    const R ex = vx[1] * vz[0] - vx[0] * vz[1];
    const R ey = vy[1] * vz[0] - vy[0] * vz[1];
    const R A = f2 * (ex * ex + ey * ey);
    const R zz = vz[0] * vz[1];
    const R z4 = zz * zz;
    const R Bs = t2s * z4;
    const R Bm = t2m * z4;
    if (A > Bs) return kSplit;
    if (A < Bm) return kMerge;
    return kKeep;
}

// vertex-cache record of block s: world positions of the three vertices,
// the depth and the heap ID
__device__ __forceinline__ void store_rec(float4* w, Vec3<float> pa, Vec3<float> pb, Vec3<float> pc, int depth,
                                          uint64_t id)
{
    w[0] = make4(pa, (uint32_t)depth);
    w[1] = make4(pb, (uint32_t)id);
    w[2] = make4(pc, (uint32_t)(id >> 32));
}

__device__ __forceinline__ void store_rec(double4* w, Vec3<double> pa, Vec3<double> pb, Vec3<double> pc, int depth,
                                          uint64_t id)
{
    w[0] = make4(pa, (uint64_t)depth);
    w[1] = make4(pb, id);
    w[2] = make4(pc, (uint64_t)0);
}

template <typename R>
__device__ __forceinline__ void store_world(const Pool& P, uint32_t s, Vec3<R> pa, Vec3<R> pb, Vec3<R> pc, int depth,
                                            uint64_t id)
{
    store_rec(world_rec<R>(P, s), pa, pb, pc, depth, id);
}

// a new bisector's vertex record, which carries its heap ID (the pointer
// pass writes its pointers)
template <typename R>
__device__ __forceinline__ void store_output(const Pool& P, uint32_t q, Vec3<R> pa, Vec3<R> pb, Vec3<R> pc, int depth,
                                             uint64_t id)
{
    store_world<R>(P, q, pa, pb, pc, depth, id);
}

// ---------------------------------------------------------------------------
// kernel: classify -> fresh command word (the vertex cache holds the world
// positions, the depth and the parity, so no heap ID is read)
// ---------------------------------------------------------------------------

// The even MERGE members are listed (block, depth) per workgroup in rank
// order: wave ballots place them, one barrier per tile exchanges the waves'
// counts per row (the vote's result does not depend on the order within the
// list; rank order keeps neighbouring threads of the vote on neighbouring
// blocks).
struct Lds_classify {
    uint32_t sh[8];
    uint32_t wcnt[2][kClassRows][kBlock / 64];
};

template <typename R>
__device__ __forceinline__ void run_classify(const Pool& P, const LodK& K, const uint8_t* inj, uint32_t blk, Lds_classify& S_)
{
    auto& sh = S_.sh;
    auto& wcnt = S_.wcnt;
    // each workgroup classifies kClassChunks consecutive rank chunks, each
    // chunk with its own partial and list
    const int maxd = 63 - P.k;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t nsplit = 0, nmerge = 0, ncand = 0, tile = 0;
    for (uint32_t rb = blk * kClassChunks; rb < (blk + 1) * kClassChunks && rb < P.G; ++rb) {
        uint32_t r0, r1;
        rank_range(P.ctr->L, P.G, rb, &r0, &r1);
        uint32_t scost = 0, nlist = 0;
        // the rank entries of the next tile are loaded while this tile's
        // records are in flight (past the chunk: block 0, in bounds, unused)
        uint32_t sn[kClassRows];
#pragma unroll
        for (int j = 0; j < kClassRows; ++j) {
            const uint32_t r = r0 + j * kBlock + threadIdx.x;
            sn[j] = r < r1 ? P.live[r] : 0u;
        }
        for (uint32_t base = r0; base < r1; base += kBlock * kClassRows, ++tile) {
            // every row's loads in flight before the first row is processed
            uint32_t sr[kClassRows], dr[kClassRows];
            T4<R> wa[kClassRows], wb[kClassRows], wc[kClassRows];
            bool cand[kClassRows];
#pragma unroll
            for (int j = 0; j < kClassRows; ++j) {
                sr[j] = sn[j];
                const T4<R>* w = world_rec<R>(P, sr[j]);
                wa[j] = w[0];
                wb[j] = w[1];
                wc[j] = w[2];
            }
#pragma unroll
            for (int j = 0; j < kClassRows; ++j) {
                const uint32_t r = base + (kClassRows + j) * kBlock + threadIdx.x;
                sn[j] = r < r1 ? P.live[r] : 0u;
            }
#pragma unroll
            for (int j = 0; j < kClassRows; ++j) {
                cand[j] = false;
                dr[j] = 0;
                const uint32_t r = base + j * kBlock + threadIdx.x;
                if (r >= r1) continue;
                const uint32_t s = sr[j];
                const int d = w_int(wa[j].w);
                dr[j] = (uint32_t)d;
                uint32_t dec;
                if (inj) {
                    dec = inj[s];
                    if (dec > kMerge) {
                        raise_err(P, kErrDecision);
                        dec = kKeep;
                    }
                } else {
                    dec = lod_decide<R>(K, ld3<R>(wa[j]), ld3<R>(wb[j]), ld3<R>(wc[j]));
                }
                if (dec == kMerge && d == 0) dec = kKeep;       // roots never merge
                if (dec == kSplit && d + 1 > maxd) dec = kKeep; // index width
                if ((uint32_t)d > 63u) {
                    raise_err(P, kErrPointer);
                    dec = kKeep;
                }
                P.cmd[s] = dec | ((uint32_t)d << kDepthShift);
                if (dec == kSplit) {
                    ++nsplit;
                    scost += 3u * (uint32_t)d + 4u;
                } else if (dec == kMerge) {
                    ++nmerge;
                    // configurations are found from their even members (Alg. 4)
                    cand[j] = (RecId<R>::low(wb[j]) & 1u) == 0;
                }
            }
            // rank order within the tile: (row, wave, lane)
            uint64_t m[kClassRows];
#pragma unroll
            for (int j = 0; j < kClassRows; ++j) {
                m[j] = __ballot(cand[j]);
                if (lane == 0) wcnt[tile & 1][j][wv] = (uint32_t)__popcll(m[j]);
            }
            __syncthreads();
            uint32_t at = r0 + nlist;
#pragma unroll
            for (int j = 0; j < kClassRows; ++j) {
                uint32_t before = 0, row = 0;
#pragma unroll
                for (int i = 0; i < kBlock / 64; ++i) {
                    const uint32_t t = wcnt[tile & 1][j][i];
                    before += i < wv ? t : 0u;
                    row += t;
                }
                if (cand[j]) P.list[at + before + lanes_below(m[j])] = make_uint2(sr[j], dr[j]);
                at += row;
            }
            nlist = at - r0;
        }
        // a chunk's split reservations can pass 2^32 in the deepest pools
        // (2^30 blocks over 16 workgroups); a saturated sum is over any F
        const uint32_t c = block_sum_sat(scost, sh);
        if (threadIdx.x == 0) {
            P.part[rb] = make_uint2(0, c);
            P.lcnt[rb] = nlist;
        }
        ncand += nlist;
    }
    const uint32_t a = block_sum(nsplit, sh);
    const uint32_t b = block_sum(nmerge, sh);
    if (threadIdx.x == 0) {
        stat_add(P, blk, kStSplitReq, a);
        stat_add(P, blk, kStMergeReq, b);
        stat_add(P, blk, kStMergeCand, ncand);
    }
}

template <bool kB, typename R>
__global__ void __launch_bounds__(kBlock) k_classify(Batch B, Inst one)
{
    __shared__ Lds_classify S_;
    Pool P;
    LodK K;
    const uint8_t* inj;
    const uint32_t blk = pick_k<kB>(B, one, B.map_rank, P, K, inj);
    run_classify<R>(P, K, inj, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: merge configurations (list of even MERGE members)
// ---------------------------------------------------------------------------

// Alg. 4 seen from an even member c0 of depth d >= 1: j2 = Next (its
// sibling), j3 = Prev; a border pair when Prev is null, a cycle of four when
// j3 has depth d and j4 = Prev(j3) is j3's sibling.  Next of an even child
// and Prev of an odd child cross their parent's interior edge, so in a
// conforming triangulation a bisector of the same depth across them is the
// sibling, and one of depth d across Prev of c0 (half of the parent's base
// edge) is the odd child of the parent's twin: the depths in the members'
// command words decide, without their heap IDs.  The smallest ID of a
// configuration is always an even member (c0 < c1), so configurations are
// detected, once, from their even members.
//
// A configuration merges only if every member decided MERGE (unanimity),
// so each member's decision is checked as soon as its command word arrives
// and the next level of loads is skipped on a refusal; the heap IDs that
// pick the smallest member of a cycle of four are loaded for unanimous
// cycles only.  Returns the configuration size (0: none that merges, or
// not found from its smallest member).
__device__ __forceinline__ int merge_vote_even(const Pool& P, uint32_t s, int d, int32_t* j2o, int32_t* j3o,
                                               int32_t* j4o)
{
    const int4 l1 = P.lf[s].l;
    const int32_t j2 = l1.y, j3 = l1.z;
    if ((j2 >= 0 && !slot_ok(P, j2)) || (j3 >= 0 && !slot_ok(P, j3))) { raise_err(P, kErrPointer); return 0; }
    if (j2 < 0) return 0;
    const uint32_t a3 = j3 >= 0 ? (uint32_t)j3 : 0u;   // in bounds either way
    const uint32_t cm2 = P.cmd[j2];
    const int32_t j4 = P.lf[a3].l.z;
    const uint32_t cm3 = P.cmd[a3];
    const auto merges = [d](uint32_t c) { return depth_of_cmd(c) == d && (c & kDecMask) == kMerge; };
    if (!merges(cm2)) return 0;
    *j2o = j2;
    if (j3 < 0) return 2;
    if (!merges(cm3) || j4 < 0) return 0;
    if (!slot_ok(P, j4)) { raise_err(P, kErrPointer); return 0; }
    const uint32_t cm4 = P.cmd[j4];
    if (!merges(cm4)) return 0;
    if (block_id(P, (uint32_t)j4) < block_id(P, s)) return 0;   // found from the cycle's smallest member
    *j3o = j3;
    *j4o = j4;
    return 4;
}

// A unanimous configuration's reservation, one block per parent, is charged
// to the smallest member (added to the partial of the rank workgroup that
// holds it).
// rank workgroups whose merge reservations a vote workgroup sums in LDS
constexpr uint32_t kVoteAcc = 8;

struct Lds_vote {
    uint32_t sh[8];
    uint32_t base[kMaxRankGroups + 1];
    uint32_t acc[kVoteAcc];
};

__device__ __forceinline__ void run_vote(const Pool& P, uint32_t blk, Lds_vote& S_)
{
    auto& sh = S_.sh;
    auto& base = S_.base;
    auto& acc = S_.acc;
    const ListShare ls = list_share(P, blk, base, sh);
    // reservations per rank workgroup: the workgroup's entries come from a
    // few consecutive rank workgroups [w0, w0 + kVoteAcc), summed in LDS and
    // added with one atomic each (many threads adding into the same partial
    // serialise); entries of later ones (tiny chunks) go straight to memory
    const uint32_t w0 = share_start(base, P.G, ls);
    uint32_t wh = w0;
    if (threadIdx.x < kVoteAcc) acc[threadIdx.x] = 0;
    __syncthreads();
    uint32_t ncfg = 0;
    for (uint32_t i = ls.i0 + threadIdx.x; i < ls.i1; i += kBlock) {
        const uint2 e = P.list[list_at_from(base, ls.chunk, i, &wh)];   // (block, depth)
        const uint32_t w = wh;
        const uint32_t s = e.x;
        int32_t j2 = -1, j3 = -1, j4 = -1;
        const int m = merge_vote_even(P, s, (int)e.y, &j2, &j3, &j4);
        if (!m) continue;
        P.cmd[s] |= kMCfg | kMMin | kMUnan | (m == 4 ? kMQuad : 0u);
        P.lf[s].f = make_uint4((uint32_t)j2, (uint32_t)j3, (uint32_t)j4, (uint32_t)m);
        if (w - w0 < kVoteAcc) atomicAdd(&acc[w - w0], (uint32_t)m / 2);
        else atomicAdd(&P.part[w].x, (uint32_t)m / 2);
        ++ncfg;
    }
    __syncthreads();
    if (threadIdx.x < kVoteAcc && acc[threadIdx.x]) atomicAdd(&P.part[w0 + threadIdx.x].x, acc[threadIdx.x]);
    const uint32_t u = block_sum(ncfg, sh);
    if (threadIdx.x == 0) stat_add(P, blk, kStMergeCfg, u);
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_vote(Batch B, Inst one)
{
    __shared__ Lds_vote S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_list, P);
    run_vote(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: reservation cut
// ---------------------------------------------------------------------------

// Rank-order cut: the merge reservation of rank r is accepted when the
// inclusive merge prefix fits in F; the split reservation (3d + 4) when all
// merge reservations plus the inclusive split prefix fit in F.  Accepted
// initiators are listed for the chain walk.
struct Lds_budget {
    uint2 sh2[8];
    uint32_t sh[8];
};

__device__ __forceinline__ void run_budget(const Pool& P, uint32_t blk, Lds_budget& S_)
{
    auto& sh2 = S_.sh2;
    auto& sh = S_.sh;
    uint32_t r0, r1;
    rank_range(P.ctr->L, P.G, blk, &r0, &r1);
    // reservations (merge, split) of the rank workgroups before this one,
    // and the merge total: every workgroup sums the partials itself
    uint2 before = make_uint2(0, 0), all = before;
    for (uint32_t g = threadIdx.x; g < P.G; g += kBlock) {
        const uint2 v = P.part[g];
        all = sat_add2(all, v);
        if (g < blk) before = sat_add2(before, v);
    }
    uint2 carry = block_reduce_sat2(before, sh2);
    const uint32_t Tm = block_reduce_sat2(all, sh2).x;
    const uint32_t F = P.ctr->F;
    uint32_t nm = 0, nlist = 0;
    uint32_t sn[kSeg];   // the next tile's segment, loaded a tile ahead
    load_seg(P, r0 + threadIdx.x * kSeg, r1, sn);
    for (uint32_t base = r0; base < r1; base += kBlock * kSeg) {
        const uint32_t t0 = base + threadIdx.x * kSeg;
        uint32_t sr[kSeg], cr[kSeg];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) sr[j] = sn[j];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) cr[j] = t0 + j < r1 ? P.cmd[sr[j]] : 0u;
        load_seg(P, t0 + kBlock * kSeg, r1, sn);
        // reservations: (merge blocks, split blocks 3d + 4) per rank
        uint2 v[kSeg];
        uint2 loc = make_uint2(0, 0);
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t c = cr[j];
            v[j] = make_uint2((c & kMUnan) ? ((c & kMQuad) ? 2u : 1u) : 0u,
                              (c & kDecMask) == kSplit ? 3u * (uint32_t)depth_of_cmd(c) + 4u : 0u);
            loc = sat_add2(loc, v[j]);
        }
        uint2 tot;
        uint2 run = sat_add2(carry, block_excl_scan_sat(loc, sh2, &tot));
        uint32_t acc = 0;   // bit j: the split reservation of rank t0 + j fits
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            run = sat_add2(run, v[j]);   // inclusive prefix at this rank
            if (v[j].x && run.x <= F) {
                P.cmd[sr[j]] = cr[j] | kMAcc;
                ++nm;
            }
            if (v[j].y && sat_add(Tm, run.y) <= F) acc |= 1u << j;
        }
        uint32_t ltot;
        uint32_t at = r0 + nlist + block_excl_scan((uint32_t)__popc(acc), sh, &ltot);
#pragma unroll
        for (int j = 0; j < kSeg; ++j)
            if ((acc >> j) & 1u) P.list[at++] = make_uint2(sr[j], 0);
        nlist += ltot;
        carry = sat_add2(carry, tot);
    }
    const uint32_t a = block_sum(nm, sh);
    if (threadIdx.x == 0) {
        P.lcnt[blk] = nlist;
        stat_add(P, blk, kStMergeAcc, a);
        stat_add(P, blk, kStSplitAcc, nlist);
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_budget(Batch B, Inst one)
{
    __shared__ Lds_budget S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_rank, P);
    run_budget(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: compatibility chains (list of accepted initiators)
// ---------------------------------------------------------------------------

// Walk from an accepted initiator through Twin: a same-level twin pair ends
// the chain; a coarser twin receives the mark of the edge it shares (Next or
// Prev) plus its own base mark and the walk continues from it.  A walk stops
// at a base mark already set: whoever set it walks (or walked) the same
// remaining chain, which depends on pre-frame pointers only.
__device__ void walk_chain(const Pool& P, uint32_t s)
{
    uint32_t old = atomicOr(&P.cmd[s], kMarkB);
    if (old & kMarkB) return;
    int32_t cur = (int32_t)s;
    for (int it = 0; it < 130; ++it) {
        const int32_t n = P.lf[cur].l.x;
        if (n < 0) return;
        if (!slot_ok(P, n)) { raise_err(P, kErrPointer); return; }
        const int4 ln = P.lf[n].l;
        if (ln.x == cur) {
            atomicOr(&P.cmd[n], kMarkB);
            return;
        }
        uint32_t e;
        if (ln.y == cur) e = kMarkN;
        else if (ln.z == cur) e = kMarkP;
        else { raise_err(P, kErrPointer); return; }
        old = atomicOr(&P.cmd[n], e | kMarkB);
        if (old & kMarkB) return;
        cur = n;
    }
    raise_err(P, kErrChain);
}

struct Lds_walk {
    uint32_t sh[8];
    uint32_t base[kMaxRankGroups + 1];
};

__device__ __forceinline__ void run_walk(const Pool& P, uint32_t blk, Lds_walk& S_)
{
    auto& sh = S_.sh;
    auto& base = S_.base;
    const ListShare ls = list_share(P, blk, base, sh, nullptr, P.G);
    uint32_t wh = share_start(base, P.G, ls);
    for (uint32_t i = ls.i0 + threadIdx.x; i < ls.i1; i += kBlock) {
        walk_chain(P, P.list[list_at_from(base, ls.chunk, i, &wh)].x);
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_walk(Batch B, Inst one)
{
    __shared__ Lds_walk S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_rank, P);   // G workgroups share the list
    run_walk(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: owners (split-marked bisectors, executing merges), their output
// counts per workgroup, and the owner list with the command words
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t split_outputs(uint32_t cmd)
{
    return 2u + ((cmd & kMarkN) ? 1u : 0u) + ((cmd & kMarkP) ? 1u : 0u);
}

// Whether a member of an accepted configuration (the smallest member's
// forwarding record: sibling, other odd, other even, size) is split-marked;
// the members' command words are loaded together.
__device__ __forceinline__ uint32_t merge_vetoed(const Pool& P, uint4 m)
{
    const bool quad = m.w == 4;
    const uint32_t a = P.cmd[m.x];
    const uint32_t b = quad ? P.cmd[m.y] : 0u;
    const uint32_t c = quad ? P.cmd[m.z] : 0u;
    return ((a | b | c) & kMarks) ? 1u : 0u;
}

struct Lds_owners {
    uint32_t sh[8];
    uint2 sh2[8];
};

__device__ __forceinline__ void run_owners(const Pool& P, uint32_t blk, Lds_owners& S_)
{
    auto& sh = S_.sh;
    auto& sh2 = S_.sh2;
    uint32_t r0, r1;
    rank_range(P.ctr->L, P.G, blk, &r0, &r1);
    uint32_t nexec = 0, nsc = 0, nfree = 0;
    uint2 run = make_uint2(0, 0);   // (owners, outputs) of earlier tiles
    uint32_t sn[kSeg];              // the next tile's segment, loaded a tile ahead
    load_seg(P, r0 + threadIdx.x * kSeg, r1, sn);
    for (uint32_t base = r0; base < r1; base += kBlock * kSeg) {
        const uint32_t t0 = base + threadIdx.x * kSeg;
        uint32_t sr[kSeg], cr[kSeg];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) sr[j] = sn[j];
#pragma unroll
        for (int j = 0; j < kSeg; ++j) cr[j] = t0 + j < r1 ? P.cmd[sr[j]] : 0u;
        load_seg(P, t0 + kBlock * kSeg, r1, sn);
        // split owners from the command word alone; an accepted merge (a
        // few per cent of the ranks) executes unless a member is split-marked
        // (splits win).  The checks of a thread's first two accepted merges
        // are issued together, so a wave waits for two levels of loads per
        // tile rather than two per rank that holds a merge in some lane;
        // further ones (rare) are checked one by one.
        uint64_t kk = 0;   // 4 bits of output count per rank
        static_assert(kSeg <= 16, "output counts of a segment in 64 bits");
        uint32_t macc = 0;
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t c = cr[j];
            if (c & kMarks) {
                kk |= (uint64_t)split_outputs(c) << (4 * j);
                ++nsc;
                ++nfree;
            } else if (c & kMAcc) {
                macc |= 1u << j;
            }
        }
        if (macc) {
            const int ja = __ffs(macc) - 1;
            const uint32_t rest = macc & (macc - 1);
            const int jb = rest ? __ffs(rest) - 1 : -1;
            uint32_t sa = 0, sb = 0;
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                sa = j == ja ? sr[j] : sa;
                sb = j == jb ? sr[j] : sb;
            }
            const uint4 ma = P.lf[sa].f;
            const uint4 mb = jb >= 0 ? P.lf[sb].f : make_uint4(0, 0, 0, 0);
            const uint32_t va = merge_vetoed(P, ma), vb = jb >= 0 ? merge_vetoed(P, mb) : 1u;
#pragma unroll
            for (int j = 0; j < kSeg; ++j) {
                if (!((macc >> j) & 1u)) continue;
                uint4 m;
                uint32_t veto;
                if (j == ja) {
                    m = ma;
                    veto = va;
                } else if (j == jb) {
                    m = mb;
                    veto = vb;
                } else {
                    m = P.lf[sr[j]].f;
                    veto = merge_vetoed(P, m);
                }
                if (!veto) {
                    cr[j] |= kMExec;
                    kk |= (uint64_t)(m.w / 2) << (4 * j);
                    ++nexec;
                    nfree += m.w;
                }
            }
        }
        uint2 loc = make_uint2(0, 0);   // (owners, outputs) of this segment
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t k = (uint32_t)(kk >> (4 * j)) & 15u;
            loc = make_uint2(loc.x + (k ? 1u : 0u), loc.y + k);
        }
        uint2 tot;
        const uint2 pre = block_excl_scan2(loc, sh2, &tot);
        uint32_t at = r0 + run.x + pre.x, outs = run.y + pre.y;
#pragma unroll
        for (int j = 0; j < kSeg; ++j) {
            const uint32_t k = (uint32_t)(kk >> (4 * j)) & 15u;
            if (k) {
                P.list[at] = make_uint2(sr[j], cr[j]);
                P.lpre[at] = outs;
                ++at;
                outs += k;
            }
        }
        run = make_uint2(run.x + tot.x, run.y + tot.y);
    }
    const uint32_t a = block_sum(nexec, sh);
    const uint32_t b = block_sum(nsc, sh);
    const uint32_t c = block_sum(nfree, sh);
    if (threadIdx.x == 0) {
        P.part[blk] = make_uint2(run.y, 0);
        P.lcnt[blk] = run.x;
        stat_add(P, blk, kStMergeExec, a);
        stat_add(P, blk, kStSplitConsumed, b);
        stat_add(P, blk, kStFrees, c);
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_owners(Batch B, Inst one)
{
    __shared__ Lds_owners S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_rank, P);
    run_owners(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: the first N free blocks (ZeroToBitID(0..N-1) of the pre-frame
// tree, Alg. 8), marked occupied; staged in LDS for coalesced writes
// ---------------------------------------------------------------------------

struct Lds_freelist {
    uint32_t sh[8];
    uint32_t stage[kBlock * 32];
    uint32_t sb;
};

__device__ __forceinline__ void run_freelist(const Pool& P, uint32_t blk, Lds_freelist& S_)
{
    auto& sh = S_.sh;
    auto& stage = S_.stage;
    auto& sb = S_.sb;
    // N = the outputs of every owner (the sum of the owners' partials)
    uint32_t n = 0;
    for (uint32_t g = threadIdx.x; g < P.G; g += kBlock) n += P.part[g].x;
    const uint32_t N = block_sum(n, sh);
    if (blk == 0 && threadIdx.x == 0) {
        P.ctr->N = N;
        if (N > P.ctr->F) raise_err(P, kErrAlloc);
    }
    const uint32_t w0 = blk * kWordsPerBlock;
    if (w0 >= P.W || N == 0) return;
    uint32_t zb = 32u * w0 - ones_before_word(P, w0, &sb);
    if (zb >= N) return;
    const uint32_t valid = word_valid(P);
    for (uint32_t it = 0; it < kWordsPerBlock; it += kBlock) {
        const uint32_t w = w0 + it + threadIdx.x;
        const uint32_t raw = (w < P.W) ? P.bits[w] : 0xffffffffu;
        const uint32_t word = raw | ~valid;   // blocks past a one-word pool read as taken
        uint32_t tot;
        uint32_t o = block_excl_scan(__popc(~word), sh, &tot);
        if (w < P.W && zb + o < N) {
            uint32_t inv = ~word, nw = raw;
            while (inv && zb + o < N) {
                const int j = __ffs(inv) - 1;
                stage[o++] = w * 32u + (uint32_t)j;
                nw |= 1u << j;
                inv &= inv - 1;
            }
            P.bits[w] = nw;
        }
        __syncthreads();
        const uint32_t take = (N - zb) < tot ? (N - zb) : tot;
        for (uint32_t i = threadIdx.x; i < take; i += kBlock) P.freel[zb + i] = stage[i];
        __syncthreads();
        zb += tot;
        if (zb >= N) break;
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_freelist(Batch B, Inst one)
{
    __shared__ Lds_freelist S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_word, P);
    run_freelist(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: fill (owner list) -- vertex-cache records of the outputs and the
// forwarding records and fates of consumed bisectors.  An owner's first
// output takes position (workgroup's output base) + (outputs of the
// workgroup's earlier owners) of the free list: the exclusive scan of the
// output counts in rank order.
// ---------------------------------------------------------------------------

// Forwarding record of a split bisector, by role:
//   0: first child (2x), or its first child (4x) when the Prev edge splits
//   1: second child of the first child (4x+1), Prev edge split only
//   2: second child (2x+1), or its first child (4x+2) when the Next edge splits
//   3: second child of the second child (4x+3), Next edge split only
// Outputs take their blocks in ascending heap-ID order.  A merged member's
// record holds its parent's block first; the smallest member's record also
// keeps the other members (second, third, fourth fields) for the pointer
// pass.

// Blocks of a split bisector's outputs by role, from its command word and
// its first position base in the free list (N blocks allocated); the
// unused roles hold 0xffffffff.  False (and the allocation flag raised)
// when the allocation does not hold them.
__device__ __forceinline__ bool split_targets(const Pool& P, uint32_t c, uint32_t base, uint32_t N, uint4* f)
{
    const bool hn = c & kMarkN, hp = c & kMarkP;
    const uint32_t cnt = 2u + (hn ? 1u : 0u) + (hp ? 1u : 0u);
    if (base + cnt > N) { raise_err(P, kErrAlloc); return false; }
    const uint32_t q0 = P.freel[base], q1 = P.freel[base + 1];
    const uint32_t q2 = cnt > 2 ? P.freel[base + 2] : 0u, q3 = cnt > 3 ? P.freel[base + 3] : 0u;
    if (q0 >= P.cap || q1 >= P.cap || q2 >= P.cap || q3 >= P.cap) { raise_err(P, kErrAlloc); return false; }
    const uint32_t no = 0xffffffffu;
    if (!hn && !hp) *f = make_uint4(q0, no, q1, no);          // 2x, 2x+1
    else if (hn && !hp) *f = make_uint4(q0, no, q1, q2);      // 2x, 4x+2, 4x+3
    else if (!hn && hp) *f = make_uint4(q1, q2, q0, no);      // 2x+1, 4x, 4x+1
    else *f = make_uint4(q0, q1, q2, q3);                     // 4x .. 4x+3
    return true;
}

template <typename R>
__device__ __forceinline__ void fill_split(const Pool& P, const LodK& K, uint32_t s, uint32_t c, uint32_t base,
                                           uint32_t N)
{
    using V = Vec3<R>;
    const bool hn = c & kMarkN, hp = c & kMarkP;
    // world positions and heap ID: the vertex record, loaded with the
    // outputs' blocks; flat vertices: the Alg. 2 decode of the ID (no memory
    // beyond the root table)
    const T4<R>* wv = world_rec<R>(P, s);
    const T4<R> ra = wv[0], rb = wv[1], rc = wv[2];
    uint4 f;
    if (!split_targets(P, c, base, N, &f)) return;
    const int d = depth_of_cmd(c);
    const uint64_t x = RecId<R>::get(rb, rc);
    V v0, v1, v2;
    decode<R>(P, x, d, v0, v1, v2);
    const V w0 = ld3<R>(ra), w1 = ld3<R>(rb), w2 = ld3<R>(rc);
    const V m = mid3(v0, v1);
    const V wm = world<R>(K, m);
    // first child (v0, v2, m), or its children (v0, m, m0) and (m, v2, m0)
    if (!hp) {
        store_output<R>(P, f.x, w0, w2, wm, d + 1, 2 * x);
    } else {
        const V m0 = mid3(v0, v2);
        const V wm0 = world<R>(K, m0);
        store_output<R>(P, f.x, w0, wm, wm0, d + 2, 4 * x);
        store_output<R>(P, f.y, wm, w2, wm0, d + 2, 4 * x + 1);
    }
    // second child (v2, v1, m), or its children (v2, m, m1) and (m, v1, m1)
    if (!hn) {
        store_output<R>(P, f.z, w2, w1, wm, d + 1, 2 * x + 1);
    } else {
        const V m1 = mid3(v2, v1);
        const V wm1 = world<R>(K, m1);
        store_output<R>(P, f.z, w2, wm, wm1, d + 2, 4 * x + 2);
        store_output<R>(P, f.w, wm, w1, wm1, d + 2, 4 * x + 3);
    }
    P.lf[s].l.w = (int)c;
    P.lf[s].f = f;
}

// Merges: the parent of the sibling pair (c0 even, c1 odd) has vertices
// (c0.v0, c1.v1, c0.v1) and heap ID c0 / 2, both read from the children's
// vertex records.
template <typename R>
__device__ __forceinline__ void fill_merge(const Pool& P, uint32_t s, uint32_t c, uint32_t base, uint32_t N)
{
    // the smallest member's record and first free block are loaded with
    // its forwarding record, the other members' records after it
    if (base + 1u > N) { raise_err(P, kErrAlloc); return; }
    const T4<R>* e0 = world_rec<R>(P, s);
    const T4<R> a0 = e0[0], b0 = e0[1], c0 = e0[2];
    uint32_t qa = P.freel[base], qb = 0xffffffffu;
    const uint4 m = P.lf[s].f;   // (sibling, other odd, other even, members)
    const bool quad = m.w == 4;
    if (quad && base + 2u > N) { raise_err(P, kErrAlloc); return; }
    if (m.x >= P.cap || (quad && (m.y >= P.cap || m.z >= P.cap))) { raise_err(P, kErrPointer); return; }
    const T4<R>* o0 = world_rec<R>(P, m.x);
    const T4<R> d0 = o0[1];
    const uint64_t ida = RecId<R>::get(b0, c0) >> 1;
    T4<R> a1 = a0, b1 = b0, c1 = c0, d1 = d0;
    uint64_t idb = 0;
    if (quad) {
        const T4<R>* e1 = world_rec<R>(P, m.z);
        const T4<R>* o1 = world_rec<R>(P, m.y);
        a1 = e1[0];
        b1 = e1[1];
        c1 = e1[2];
        d1 = o1[1];
        idb = RecId<R>::get(b1, c1) >> 1;
    }
    if (quad) {
        const uint32_t q1 = P.freel[base + 1];
        const bool a_first = ida < idb;
        qb = a_first ? q1 : qa;
        qa = a_first ? qa : q1;
    }
    if (qa >= P.cap || (quad && qb >= P.cap)) { raise_err(P, kErrAlloc); return; }
    const int dp = depth_of_cmd(c) - 1;
    store_output<R>(P, qa, ld3<R>(a0), ld3<R>(d0), ld3<R>(b0), dp, ida);
    P.lf[s].l.w = (int)kMExec;
    P.lf[s].f = make_uint4(qa, m.x, m.y, m.z);
    P.lf[m.x].l.w = (int)kMExec;
    P.lf[m.x].f = make_uint4(qa, 0, 0, 0);
    if (quad) {
        store_output<R>(P, qb, ld3<R>(a1), ld3<R>(d1), ld3<R>(b1), dp, idb);
        P.lf[m.y].l.w = (int)kMExec;
        P.lf[m.y].f = make_uint4(qb, 0, 0, 0);
        P.lf[m.z].l.w = (int)kMExec;
        P.lf[m.z].f = make_uint4(qb, 0, 0, 0);
    }
}

// One loop step of a workgroup over the owner list regroups its items so
// that split owners take the lowest threads (in list order), then merges,
// then empty items: each wave then runs one of the two item paths (but the
// wave at the boundary) instead of both one after the other.  An item is
// (block, command word, first free-list position).  Every thread of the
// workgroup calls this; returns whether this thread holds an item.
struct OwnerStage {
    uint32_t cnt[2][kBlock / 64];
    uint4 item[kBlock];
};

__device__ __forceinline__ bool group_owners(OwnerStage& st, bool valid, uint3& it)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool split = valid && (it.y & kMarks);
    const bool merge = valid && !(it.y & kMarks);
    const uint64_t ms = __ballot(split), mm = __ballot(merge);
    if (lane == 0) {
        st.cnt[0][wv] = (uint32_t)__popcll(ms);
        st.cnt[1][wv] = (uint32_t)__popcll(mm);
    }
    __syncthreads();
    uint32_t ps = 0, ts = 0, pm = 0, tm = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        const uint32_t a = st.cnt[0][i], b = st.cnt[1][i];
        ps += i < wv ? a : 0u;
        pm += i < wv ? b : 0u;
        ts += a;
        tm += b;
    }
    if (split) st.item[ps + lanes_below(ms)] = make_uint4(it.x, it.y, it.z, 0);
    if (merge) st.item[ts + pm + lanes_below(mm)] = make_uint4(it.x, it.y, it.z, 0);
    __syncthreads();
    const bool got = threadIdx.x < ts + tm;
    if (got) {
        const uint4 v = st.item[threadIdx.x];
        it = make_uint3(v.x, v.y, v.z);
    }
    __syncthreads();   // the stage is reused by the next step
    return got;
}

// the owner-list item of entry i of this workgroup's share
__device__ __forceinline__ uint3 owner_item(const Pool& P, const uint32_t* base, const uint32_t* obase, uint32_t chunk,
                                            uint32_t i, uint32_t* wh)
{
    const uint32_t at = list_at_from(base, chunk, i, wh);
    const uint2 e = P.list[at];
    return make_uint3(e.x, e.y, obase[*wh] + P.lpre[at]);
}

struct Lds_fill {
    uint32_t sh[8];
    uint32_t base[kMaxRankGroups + 1];
    uint32_t obase[kMaxRankGroups + 1];
    OwnerStage st;
};

template <typename R>
__device__ __forceinline__ void run_fill(const Pool& P, const LodK& K, const uint8_t* inj, uint32_t blk, Lds_fill& S_)
{
    auto& sh = S_.sh;
    auto& base = S_.base;
    auto& obase = S_.obase;
    auto& st = S_.st;
    (void)inj;
    const ListShare ls = list_share(P, blk, base, sh, obase);
    // outputs past the free blocks (an over-committed frame, flagged by the
    // free-list pass) are refused, so free-list reads stay below F
    const uint32_t N = min(obase[P.G], P.ctr->F);
    uint32_t wh = share_start(base, P.G, ls);
    for (uint32_t i0 = ls.i0; i0 < ls.i1; i0 += kBlock) {   // uniform trip count
        const uint32_t i = i0 + threadIdx.x;
        uint3 it = make_uint3(0, 0, 0);
        if (i < ls.i1) it = owner_item(P, base, obase, ls.chunk, i, &wh);
        if (!group_owners(st, i < ls.i1, it)) continue;
        if (it.y & kMarks) fill_split<R>(P, K, it.x, it.y, it.z, N);
        else fill_merge<R>(P, it.x, it.y, it.z, N);
    }
}

template <bool kB, typename R>
__global__ void __launch_bounds__(kBlock) k_fill(Batch B, Inst one)
{
    __shared__ Lds_fill S_;
    Pool P;
    LodK K;
    const uint8_t* inj;
    const uint32_t blk = pick_k<kB>(B, one, B.map_list, P, K, inj);
    run_fill<R>(P, K, inj, blk, S_);
}

// ---------------------------------------------------------------------------
// kernel: heap IDs and neighbour pointers of the new bisectors (Table 1,
// Alg. 5/6 and their compositions)
// ---------------------------------------------------------------------------

enum { kEdgeT = 0, kEdgeN = 1, kEdgeP = 2 };
enum { kWhole = 0, kHalf0 = 1, kHalf1 = 2 };   // half at the edge's first / second endpoint

// Output role of a split bisector covering (a half of) one of its old edges.
// Edges are (v0,v1), (v1,v2), (v2,v0); halves are named by the endpoint
// they contain, in that order.
__device__ __forceinline__ int cover_role(uint32_t marks, int edge, int piece)
{
    const bool n = marks & kMarkN, p = marks & kMarkP;
    if (edge == kEdgeT) {
        if (piece == kHalf0) return 0;          // first child (or its first child)
        if (piece == kHalf1) return n ? 3 : 2;  // second child (or its second child)
        return -1;
    }
    if (edge == kEdgeN) {
        if (n) return piece == kHalf0 ? 3 : (piece == kHalf1 ? 2 : -1);
        return piece == kWhole ? 2 : -1;
    }
    if (p) return piece == kHalf0 ? 1 : (piece == kHalf1 ? 0 : -1);
    return piece == kWhole ? 0 : -1;
}

__device__ __forceinline__ uint32_t comp(uint4 v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// The old neighbour across one edge of a consumed bisector b, loaded once
// (one record line): its block, which of its fields pointed to b, its fate
// this frame (0 when untouched) and its forwarding record.
struct Nb {
    int32_t n;
    int f;
    uint32_t c;
    uint4 fw;
};

// The neighbours n[i] of bisectors b[i] (-1: border), in two rounds of
// loads: the pointer records of all of them, then the forwarding records of
// those consumed this frame.  Unused slots load block 0 (in bounds, ignored).
template <int N>
__device__ __forceinline__ void load_nbs(const Pool& P, const int32_t (&b)[N], const int32_t (&n)[N], Nb (&r)[N])
{
    int4 ln[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const bool ok = slot_ok(P, n[i]);
        if (n[i] >= 0 && !ok) raise_err(P, kErrPointer);
        ln[i] = P.lf[ok ? n[i] : 0].l;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const bool ok = slot_ok(P, n[i]);
        const int f = ln[i].x == b[i] ? 0 : (ln[i].y == b[i] ? 1 : (ln[i].z == b[i] ? 2 : -1));
        if (ok && f < 0) raise_err(P, kErrPointer);
        const bool use = ok && f >= 0;
        r[i].n = use ? n[i] : -1;
        r[i].f = f;
        r[i].c = use ? (uint32_t)ln[i].w : 0u;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) r[i].fw = P.lf[r[i].c ? r[i].n : 0].f;
}

// New neighbour across (a piece of) an old edge, seen from output x: the
// untouched neighbour itself (whose back-pointer x then takes over -- its
// only writer), the output of a split neighbour covering the same piece
// (halves swap names between bisectors of equal depth and keep them across a
// depth difference of one), or a merged neighbour's parent.
__device__ __forceinline__ int32_t piece_target(const Pool& P, const Nb& nb, int db, int piece, uint32_t x)
{
    if (nb.n < 0) return -1;
    if (nb.c & kMarks) {
        int pn = piece;
        if (piece != kWhole && depth_of_cmd(nb.c) == db) pn = piece == kHalf0 ? kHalf1 : kHalf0;
        const int role = cover_role(nb.c & kMarks, nb.f, pn);
        if (role < 0) { raise_err(P, kErrEdge); return -1; }
        return (int32_t)comp(nb.fw, role);
    }
    if (nb.c & kMExec) return (int32_t)nb.fw.x;
    if (piece != kWhole) { raise_err(P, kErrEdge); return -1; }
    reinterpret_cast<int*>(&P.lf[nb.n].l)[nb.f] = (int)x;
    return nb.n;
}

// a new bisector's pointers and untouched fate (the fill wrote its heap ID)
__device__ __forceinline__ void store_new(const Pool& P, uint32_t q, int32_t t, int32_t n, int32_t p)
{
    if (q >= P.cap) { raise_err(P, kErrAlloc); return; }
    P.lf[q].l = make_int4(t, n, p, 0);
}

// Bits of consumed bisectors to clear, at most two bitfield words per work
// item (a split bisector; or the two sibling pairs of a merge, each pair
// usually in one word).  kNoWord: nothing.  Device-wide atomics are
// expensive on a multi-die GPU (each goes past the die's L2), so the lanes
// of a wave first merge the masks of equal words and one lane per word
// clears them.
constexpr uint32_t kNoWord = 0xffffffffu;
struct Clears {
    uint32_t w[2], m[2];
};

__device__ __forceinline__ void add_clear(const Pool& P, Clears& c, int slot, uint32_t s)
{
    const uint32_t w = s >> 5, m = 1u << (s & 31u);
    if (c.w[slot] == kNoWord) {
        c.w[slot] = w;
        c.m[slot] = m;
    } else if (c.w[slot] == w) {
        c.m[slot] |= m;
    } else {
        atomicAnd(&P.bits[w], ~m);   // a pair split across two words
    }
}

// Every lane of the wave calls this (convergent): a segmented OR over
// neighbouring lanes with the same word, then one atomic per run of lanes.
__device__ __forceinline__ void clear_bits_wave(const Pool& P, uint32_t w, uint32_t m)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t wo = __shfl_down(w, o, 64), mo = __shfl_down(m, o, 64);
        if (lane + o < 64 && wo == w) m |= mo;
    }
    const uint32_t wp = __shfl_up(w, 1, 64);
    if (w != kNoWord && (lane == 0 || wp != w)) atomicAnd(&P.bits[w], ~m);
}

__device__ __forceinline__ void resolve_split(const Pool& P, int32_t b, uint32_t c, uint32_t base, uint32_t N,
                                              Clears& cl)
{
    const int db = depth_of_cmd(c);
    const bool hn = c & kMarkN, hp = c & kMarkP;
    const int4 lb = P.lf[b].l;   // loaded with the outputs' blocks
    uint4 f;   // the outputs' blocks, from the free list as the fill took them
    if (!split_targets(P, c, base, N, &f)) return;
    const int32_t own[3] = {b, b, b};
    const int32_t across[3] = {lb.x, lb.y, lb.z};
    Nb nb[3];
    load_nbs(P, own, across, nb);
    const Nb& nT = nb[0];
    const Nb& nN = nb[1];
    const Nb& nP = nb[2];
    if (!hp) {  // first child (v0, v2, m)
        store_new(P, f.x, piece_target(P, nP, db, kWhole, f.x), (int32_t)f.z,
                  piece_target(P, nT, db, kHalf0, f.x));
    } else {    // its two children
        store_new(P, f.x, piece_target(P, nT, db, kHalf0, f.x), (int32_t)f.y,
                  piece_target(P, nP, db, kHalf1, f.x));
        store_new(P, f.y, (int32_t)f.z, piece_target(P, nP, db, kHalf0, f.y), (int32_t)f.x);
    }
    if (!hn) {  // second child (v2, v1, m)
        store_new(P, f.z, piece_target(P, nN, db, kWhole, f.z), piece_target(P, nT, db, kHalf1, f.z),
                  (int32_t)(hp ? f.y : f.x));
    } else {    // its two children
        store_new(P, f.z, (int32_t)(hp ? f.y : f.x), (int32_t)f.w, piece_target(P, nN, db, kHalf1, f.z));
        store_new(P, f.w, piece_target(P, nT, db, kHalf1, f.w), piece_target(P, nN, db, kHalf0, f.w),
                  (int32_t)f.z);
    }
    add_clear(P, cl, 0, (uint32_t)b);
}

// Parents of an executed merge (owner b, the smallest member): a parent q of
// the sibling pair (c0 even, c1 odd) has Next edge = c1's base edge, Prev
// edge = c0's base edge and Twin = the other parent (or the border).  The
// members' pointer records, then their base-edge neighbours, are loaded in
// one round each; a border pair loads its own members twice (unused).
__device__ __forceinline__ void resolve_merge(const Pool& P, int32_t b, uint32_t c, Clears& cl)
{
    const uint4 f = P.lf[b].f;   // (parent, sibling, other odd, other even)
    const int d = depth_of_cmd(c);
    const bool quad = (c & kMQuad) != 0;
    // a record the fill did not rewrite (its allocation failed) is refused
    if (f.x >= P.cap || f.y >= P.cap || (quad && (f.z >= P.cap || f.w >= P.cap))) {
        raise_err(P, kErrAlloc);
        return;
    }
    const uint32_t e2 = quad ? f.w : (uint32_t)b, o2 = quad ? f.z : f.y;
    const uint32_t qb = P.lf[e2].f.x;            // the second parent
    const int32_t mem[4] = {(int32_t)f.y, b, (int32_t)o2, (int32_t)e2};
    const int32_t twin[4] = {P.lf[f.y].l.x, P.lf[b].l.x, P.lf[o2].l.x, P.lf[e2].l.x};
    Nb nb[4];
    load_nbs(P, mem, twin, nb);
    store_new(P, f.x, quad ? (int32_t)qb : -1, piece_target(P, nb[0], d, kWhole, f.x),
              piece_target(P, nb[1], d, kWhole, f.x));
    if (quad) {
        store_new(P, qb, (int32_t)f.x, piece_target(P, nb[2], d, kWhole, qb), piece_target(P, nb[3], d, kWhole, qb));
        add_clear(P, cl, 1, f.z);
        add_clear(P, cl, 1, f.w);
    }
    add_clear(P, cl, 0, (uint32_t)b);
    add_clear(P, cl, 0, f.y);
}

struct Lds_resolve {
    uint32_t sh[8];
    uint32_t base[kMaxRankGroups + 1];
    uint32_t obase[kMaxRankGroups + 1];
    OwnerStage st;
};

__device__ __forceinline__ void run_resolve(const Pool& P, uint32_t blk, Lds_resolve& S_)
{
    auto& sh = S_.sh;
    auto& base = S_.base;
    auto& obase = S_.obase;
    auto& st = S_.st;
    // the owner list shared over all G rank workgroups (twice the other list
    // passes: its scattered writes and dependent record loads want more
    // waves in flight, 124 against 130 us per terrain frame)
    const ListShare ls = list_share(P, blk, base, sh, obase, P.G);
    // outputs past the free blocks (an over-committed frame, flagged by the
    // free-list pass) are refused, so free-list reads stay below F
    const uint32_t N = min(obase[P.G], P.ctr->F);
    uint32_t wh = share_start(base, P.G, ls);
    // uniform trip count: items are regrouped across the workgroup and the
    // bit clears merged across the wave
    for (uint32_t i0 = ls.i0; i0 < ls.i1; i0 += kBlock) {
        const uint32_t i = i0 + threadIdx.x;
        uint3 it = make_uint3(0, 0, 0);
        if (i < ls.i1) it = owner_item(P, base, obase, ls.chunk, i, &wh);
        const bool got = group_owners(st, i < ls.i1, it);
        Clears cl = {{kNoWord, kNoWord}, {0u, 0u}};
        if (got) {
            if (it.y & kMarks) resolve_split(P, (int32_t)it.x, it.y, it.z, N, cl);
            else resolve_merge(P, (int32_t)it.x, it.y, cl);
        }
        clear_bits_wave(P, cl.w[0], cl.m[0]);
        clear_bits_wave(P, cl.w[1], cl.m[1]);
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_resolve(Batch B, Inst one)
{
    __shared__ Lds_resolve S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_rank, P);
    run_resolve(P, blk, S_);
}

// ---------------------------------------------------------------------------
// kernels: sum-reduction tree (down to the word level; the levels below a
// word are popcounts of the bitfield and are never stored)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int sub_levels(const Pool& P)
{
    const int LW = word_level(P.D);
    return LW < P.sub ? LW : P.sub;
}

struct Lds_reduce_sub {
    uint32_t buf[2][1 << kMaxReduceSub];
};

__device__ __forceinline__ void run_reduce_sub(const Pool& P, uint32_t blk, Lds_reduce_sub& S_)
{
    auto& buf = S_.buf;
    const int LW = word_level(P.D);
    const int SUB = sub_levels(P);
    const uint32_t wpb = 1u << SUB;
    const uint32_t w0 = blk * wpb;
    const uint32_t valid = word_valid(P);
    for (uint32_t i = threadIdx.x; i < wpb; i += kBlock) {
        const uint32_t c = __popc(P.bits[w0 + i] & valid);
        buf[0][i] = c;
        P.tree[(1u << LW) + w0 + i] = c;
    }
    __syncthreads();
    int src = 0;
    for (int lvl = 1; lvl <= SUB; ++lvl) {
        const uint32_t n = wpb >> lvl;
        for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
            const uint32_t v = buf[src][2 * i] + buf[src][2 * i + 1];
            buf[src ^ 1][i] = v;
            P.tree[(1u << (LW - lvl)) + (blk << (SUB - lvl)) + i] = v;
        }
        __syncthreads();
        src ^= 1;
    }
}

template <bool kB>
__global__ void __launch_bounds__(kBlock) k_reduce_sub(Batch B, Inst one)
{
    __shared__ Lds_reduce_sub S_;
    Pool P;
    const uint32_t blk = pick<kB>(B, one, B.map_red, P);
    run_reduce_sub(P, blk, S_);
}

// the levels above the workgroup subtrees (one workgroup per instance)
__device__ __forceinline__ void run_reduce_top(const Pool& P)
{
    const int top = word_level(P.D) - sub_levels(P);   // levels [0, top) remain
    for (int lvl = top - 1; lvl >= 0; --lvl) {
        const uint32_t n = 1u << lvl;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t node = n + i;
            P.tree[node] = P.tree[2 * node] + P.tree[2 * node + 1];
        }
        __syncthreads();
    }
    // the frame statistics: each thread folds and clears one statistic's
    // lanes (the passes that add to them have completed)
    if (threadIdx.x < (uint32_t)kStCount) {
        uint32_t v[kStLanes];
#pragma unroll
        for (int l = 0; l < kStLanes; ++l) v[l] = P.slane[l * kLaneWords + threadIdx.x];
        uint32_t sum = 0;
#pragma unroll
        for (int l = 0; l < kStLanes; ++l) {
            sum += v[l];
            P.slane[l * kLaneWords + threadIdx.x] = 0u;
        }
        P.ctr->stat[threadIdx.x] = sum;
    }
}

template <bool kB>
__global__ void __launch_bounds__(1024) k_reduce_top(Batch B, Inst one)
{
    Pool P;
    pick_inst<kB>(B, one, P);
    run_reduce_top(P);
}

// ---------------------------------------------------------------------------
// persistent batched frame: the whole pipeline of every member instance in
// one launch.  The work items (phase, instance, workgroup of that
// instance's grid for the phase) are numbered phase by phase; resident
// workgroups take them in increasing order from one ticket counter.  An
// item of phase p waits until every item of phase p - 1 of its own
// instance has finished (a per-instance counter per phase), so instances
// move through the pipeline at their own pace: a small instance's later
// phases run while a large one is still in an early phase, and no phase
// ends in a device-wide drain.  An item depends only on items with smaller
// numbers, which were handed to workgroups already running, so the waits
// always end; each is also bounded (kSpinLimit polls), after which the
// item is skipped and the instance's error flag raised.
// ---------------------------------------------------------------------------

// workgroups of instance P's grid in phase ph
__device__ __forceinline__ uint32_t phase_groups(const Pool& P, int ph)
{
    switch (ph) {
    case kPhEnum:
    case kPhFree: return (P.W + kWordsPerBlock - 1) / kWordsPerBlock;
    case kPhVote:
    case kPhFill: return list_groups(P);
    case kPhClass:
    case kPhBudget:
    case kPhWalk:
    case kPhOwners:
    case kPhResolve: return P.G;
    case kPhRedSub: return P.W >> sub_levels(P);
    default: return 1u;
    }
}

// work items of one instance's phase, at most
constexpr uint32_t kPersistItems = 64;

// Each item of the persistent frame runs a span of consecutive workgroups
// of its instance's grid for the phase, so that a phase of an instance is
// at most kPersistItems items: the synchronisation a work item pays (one
// L2 write-back on its die, one counter update) is paid per span.
__device__ __forceinline__ uint32_t persist_span(uint32_t groups)
{
    return (groups + kPersistItems - 1) / kPersistItems;
}

__device__ __forceinline__ uint32_t persist_items(uint32_t groups)
{
    const uint32_t sp = persist_span(groups);
    return (groups + sp - 1) / sp;
}

union LdsAny {
    Lds_enumerate e;
    Lds_classify c;
    Lds_vote v;
    Lds_budget b;
    Lds_walk w;
    Lds_owners o;
    Lds_freelist f;
    Lds_fill fl;
    Lds_resolve r;
    Lds_reduce_sub rs;
};

// polls of one wait (a few microseconds each): about two seconds, far
// beyond any phase of a depth-30 instance
constexpr uint32_t kSpinLimit = 1u << 20;
// consecutive work items a workgroup takes per ticket
constexpr uint32_t kPersistChunk = 4;

// The loop state lives in LDS (the launch arguments are copied there once
// and each item's decode is kept there), so nothing but the LDS base stays
// in registers across a phase body: the bodies get the registers they have
// as separate kernels.
//
// Synchronisation costs are what decide this kernel on a GPU of several
// dies: an agent-scope acquire invalidates the die's L2 and an agent-scope
// release writes it back.  So the waits poll with plain coherent loads and
// acquire once, a finished item releases once (every wave first waits for
// its own stores, then one thread writes the L2 back and counts the item),
// and a workgroup takes kPersistChunk consecutive items per ticket.
struct PersistState {
    Batch B;
    Persist W;
    uint32_t item, end, inst, blk, ph, go;
};

template <typename R>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
k_persist(Batch B, Persist W)
{
    __shared__ LdsAny S_;
    __shared__ PersistState Z;
    if (threadIdx.x == 0) {
        Z.B = B;
        Z.W = W;
        Z.item = 0;
        Z.end = 0;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t item = Z.item + 1;
            if (item >= Z.end) {
                item = atomicAdd(Z.W.ticket, kPersistChunk);
                Z.end = item + kPersistChunk;
            }
            Z.item = item;
            if (item < Z.W.first[kPhCount]) {
                int ph = 0;
                uint32_t f = 0;   // first[0] = 0
                for (int q = 1; q < kPhCount; ++q) {
                    if (item >= Z.W.first[q]) {
                        ph = q;
                        f = Z.W.first[q];
                    }
                }
                (void)f;
                const uint32_t e = Z.W.map[item];
                const uint32_t in = e >> kMapShift;
                Z.inst = in;
                Z.blk = e & ((1u << kMapShift) - 1u);   // the span's index
                Z.ph = (uint32_t)ph;
                uint32_t go = 1;
                if (ph > 0) {
                    // the previous phase of this instance has finished
                    const Pool& Pq = Z.B.inst[in].P;
                    const uint32_t want = persist_items(phase_groups(Pq, ph - 1));
                    const uint32_t* dp = Z.W.done + (size_t)in * kPhCount + (ph - 1);
                    const uint32_t* ep = &Pq.ctr->err;
                    uint32_t n = 0;
                    // a stage the host marked (test hook) gives up at once,
                    // as if its wait had run out
                    if ((uint32_t)ph == Z.W.fail_phase) n = kSpinLimit;
                    while (n >= kSpinLimit ||
                           __hip_atomic_load(dp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                        // give up after kSpinLimit polls, or at once when an
                        // earlier wait of this instance gave up
                        if (++n >= kSpinLimit ||
                            (__hip_atomic_load(ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrSpin)) {
                            raise_err(Pq, kErrSpin);
                            go = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    // once a wait of this instance has given up, none of its
                    // later stages runs (their inputs would be incomplete)
                    if (__hip_atomic_load(ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrSpin) go = 0;
                    // one acquire for the whole wait: the die's caches
                    // are invalidated once the earlier phase is complete
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                Z.go = go;
            }
        }
        __syncthreads();
        // uniform values: the bodies see their instance through scalar loads
        const uint32_t item = __builtin_amdgcn_readfirstlane(Z.item);
        if (item >= Z.W.first[kPhCount]) break;
        if (__builtin_amdgcn_readfirstlane(Z.go)) {
            const Inst* I = B.inst + __builtin_amdgcn_readfirstlane(Z.inst);
            const uint32_t ph = __builtin_amdgcn_readfirstlane(Z.ph);
            const uint32_t groups = phase_groups(I->P, (int)ph);
            const uint32_t sp = persist_span(groups);
            const uint32_t b0 = __builtin_amdgcn_readfirstlane(Z.blk) * sp;
            const uint32_t b1 = b0 + sp < groups ? b0 + sp : groups;
            for (uint32_t blk = b0; blk < b1; ++blk) {
            if (blk > b0) __syncthreads();   // the previous body's LDS reads are done
            // each body loads its instance through its own opaque copy of
            // the pointer, so no load is shared between bodies and hoisted
            // above the switch (which would keep it live through every body)
#define CBT_OPAQUE(J) const Inst* J = I; asm volatile("" : "+s"(J))
            switch (ph) {
            case kPhEnum: { CBT_OPAQUE(J); run_enumerate(J->P, blk, S_.e); } break;
            case kPhClass: { CBT_OPAQUE(J); run_classify<R>(J->P, J->K, J->inj, blk, S_.c); } break;
            case kPhVote: { CBT_OPAQUE(J); run_vote(J->P, blk, S_.v); } break;
            case kPhBudget: { CBT_OPAQUE(J); run_budget(J->P, blk, S_.b); } break;
            case kPhWalk: { CBT_OPAQUE(J); run_walk(J->P, blk, S_.w); } break;
            case kPhOwners: { CBT_OPAQUE(J); run_owners(J->P, blk, S_.o); } break;
            case kPhFree: { CBT_OPAQUE(J); run_freelist(J->P, blk, S_.f); } break;
            case kPhFill: { CBT_OPAQUE(J); run_fill<R>(J->P, J->K, J->inj, blk, S_.fl); } break;
            case kPhResolve: { CBT_OPAQUE(J); run_resolve(J->P, blk, S_.r); } break;
            case kPhRedSub: { CBT_OPAQUE(J); run_reduce_sub(J->P, blk, S_.rs); } break;
            default: { CBT_OPAQUE(J); run_reduce_top(J->P); } break;
            }
#undef CBT_OPAQUE
            }
        }
        // every wave's memory operations complete (its stores in the L2)
        // before the barrier; then one release writes the L2 back and the
        // item is counted
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(Z.W.done + (size_t)Z.inst * kPhCount + Z.ph, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ticket and phase counters of a persistent frame -> zero
__global__ void k_persist_clear(Persist W, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *W.ticket = 0;
    if (i < n) W.done[i] = 0;
}

// ---------------------------------------------------------------------------
// kernels: vertex-cache refresh, queries, snapshot and restore
// ---------------------------------------------------------------------------

// Rebuild the cache of every live block: world positions of the Alg. 2
// decode of its heap ID, taken from the ID array (after an initialisation
// or an import, which write it) or from the block's own record (new world
// parameters between frames).
template <typename R>
__device__ __forceinline__ void run_refresh(const Pool& P, const LodK& K, const uint8_t* inj, uint32_t blk,
                                            bool from_ids)
{
    (void)inj;
    const uint32_t L = P.ctr->L;
    for (uint32_t r = blk * kBlock + threadIdx.x; r < L; r += P.G * kBlock) {
        const uint32_t s = P.live[r];
        const uint64_t id = from_ids ? P.id[s] : block_id(P, s);
        Vec3<R> a = {0, 0, 0}, b = a, c = a;
        int d = 0;
        if (valid_id(P, id)) {
            d = ilog2_64(id) - P.k;
            decode<R>(P, id, d, a, b, c);
        } else {
            raise_err(P, kErrPointer);
        }
        store_world<R>(P, s, world<R>(K, a), world<R>(K, b), world<R>(K, c), d, id);
    }
}

template <bool kB, typename R>
__global__ void __launch_bounds__(kBlock) k_refresh(Batch B, Inst one, bool from_ids)
{
    Pool P;
    LodK K;
    const uint8_t* inj;
    const uint32_t blk = pick_k<kB>(B, one, B.map_rank, P, K, inj);
    run_refresh<R>(P, K, inj, blk, from_ids);
}

// Clears a pool before it is filled: heap IDs, pointer and forwarding
// records, command words, the per-workgroup partials and list lengths and
// the counters, in one launch.  The rank, free and work lists and the
// vertex cache are written before they are read in every frame and are
// left as they are.
__global__ void k_clear_pool(Pool P)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < P.cap; s += stride) {
        P.id[s] = 0;
        P.lf[s].l = make_int4(0, 0, 0, 0);
        P.lf[s].f = make_uint4(~0u, ~0u, ~0u, ~0u);
        P.cmd[s] = 0;
    }
    if (blockIdx.x == 0) {
        for (uint32_t g = threadIdx.x; g < (uint32_t)kMaxRankGroups; g += blockDim.x) {
            P.lcnt[g] = 0;
            P.part[g] = make_uint2(0, 0);
        }
        for (uint32_t i = threadIdx.x; i < (uint32_t)(kStLanes * kLaneWords); i += blockDim.x) P.slane[i] = 0u;
        if (threadIdx.x == 0) *P.ctr = Counters{};
    }
}

// The frame's accumulators that must start at zero (list lengths, partial
// sums, statistics lanes) -> cleared, for frame scratch that another
// instance's frame may have used last.
__global__ void k_clear_frame_scratch(Pool P)
{
    for (uint32_t g = threadIdx.x; g < (uint32_t)kMaxRankGroups; g += blockDim.x) {
        P.lcnt[g] = 0;
        P.part[g] = make_uint2(0, 0);
    }
    for (uint32_t i = threadIdx.x; i < (uint32_t)(kStLanes * kLaneWords); i += blockDim.x) P.slane[i] = 0u;
}

__global__ void k_bits_from_ids(Pool P)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= P.W) return;
    const uint32_t n = P.cap - w * 32u < 32u ? P.cap - w * 32u : 32u;   // a one-word pool holds fewer
    uint32_t word = 0;
    for (uint32_t j = 0; j < n; ++j)
        if (P.id[w * 32u + j] != 0) word |= 1u << j;
    P.bits[w] = word;
}

__global__ void k_gather_ids(Pool P, uint32_t r0, uint32_t n, uint64_t* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = block_id(P, P.live[r0 + i]);
}

// The bisector of rank r0 + i in the paper's notation b_j^d: its root
// halfedge and its subdivision code (a leading 1, then the d path bits).
__global__ void k_gather_canonical(Pool P, uint32_t r0, uint32_t n, int32_t* root_h, uint64_t* code)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t id = block_id(P, P.live[r0 + i]);
    int32_t h = -1;
    uint64_t c = 0;
    if (valid_id(P, id)) {
        const int d = ilog2_64(id) - P.k;
        h = (int32_t)((int64_t)(id >> d) - ((int64_t)1 << P.k));
        const uint64_t one = 1ull << d;
        c = one | (id & (one - 1ull));
    } else {
        raise_err(P, kErrPointer);
    }
    if (root_h) root_h[i] = h;
    if (code) code[i] = c;
}

__global__ void k_gather_links(Pool P, uint32_t r0, uint32_t n, int32_t* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 l = P.lf[P.live[r0 + i]].l;
    out[3 * (size_t)i + 0] = l.x;
    out[3 * (size_t)i + 1] = l.y;
    out[3 * (size_t)i + 2] = l.z;
}

// flat-domain vertices: the Alg. 2 decode of the heap ID in the instance's
// precision R, written as O (binary64 results rounded once when O is float)
template <typename R, typename O>
__global__ void k_gather_vertices(Pool P, uint32_t r0, uint32_t n, O* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t id = block_id(P, P.live[r0 + i]);
    Vec3<R> v[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (valid_id(P, id)) decode<R>(P, id, ilog2_64(id) - P.k, v[0], v[1], v[2]);
    else raise_err(P, kErrPointer);
    O* o = out + 9 * (size_t)i;
    for (int j = 0; j < 3; ++j) {
        o[3 * j + 0] = (O)v[j].x;
        o[3 * j + 1] = (O)v[j].y;
        o[3 * j + 2] = (O)v[j].z;
    }
}

__global__ void k_fill_bytes(uint8_t* out, uint32_t n, uint8_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void k_gather_decisions(Pool P, uint32_t L, uint8_t* out)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= L) return;
    const uint32_t s = P.live[r];
    out[s] = (uint8_t)(P.cmd[s] & kDecMask);
}

__global__ void k_export_heap(Pool P, uint32_t* out)
{
    const uint64_t total = 2ull * P.cap;
    const int LW = word_level(P.D);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i == 0) { out[0] = 0; continue; }
        const int lvl = ilog2_64(i);
        if (lvl <= LW) {
            out[i] = P.tree[i];
        } else {
            const uint32_t span = 1u << (P.D - lvl);
            const uint64_t first = (i - (1ull << lvl)) * span;
            const uint32_t word = P.bits[first >> 5];
            const uint32_t sh = (uint32_t)(first & 31u);
            const uint32_t mask = span == 32 ? 0xffffffffu : (((1u << span) - 1u) << sh);
            out[i] = __popc(word & mask);
        }
    }
}

__global__ void k_export_records(Pool P, uint32_t b0, uint32_t n, uint32_t* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t id = block_id(P, b0 + i);   // meaningful for live blocks only
    const int4 l = P.lf[b0 + i].l;
    uint32_t* o = out + 5 * (size_t)i;
    o[0] = (uint32_t)id;
    o[1] = (uint32_t)(id >> 32);
    o[2] = (uint32_t)l.x;
    o[3] = (uint32_t)l.y;
    o[4] = (uint32_t)l.z;
}

__global__ void k_import_records(Pool P, uint32_t b0, uint32_t n, const uint32_t* in)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* v = in + 5 * (size_t)i;
    P.id[b0 + i] = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
    P.lf[b0 + i].l = make_int4((int32_t)v[2], (int32_t)v[3], (int32_t)v[4], 0);
    P.lf[b0 + i].f = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
}

// Heap IDs of the live blocks copied from their vertex records into the ID
// array, for an export whose output overwrites the vertex cache.
__global__ void k_ids_from_records(Pool P, uint32_t L)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= L) return;
    const uint32_t s = P.live[r];
    P.id[s] = block_id(P, s);
}

// Live records, rank order: (block, id low, id high, twin, next, prev); the
// IDs from the vertex records, or from the ID array (from_ids: after
// k_ids_from_records, when the output lies in the vertex cache).
__global__ void k_export_live(Pool P, uint32_t L, uint32_t* out, bool from_ids)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= L) return;
    const uint32_t s = P.live[r];
    const uint64_t id = from_ids ? P.id[s] : block_id(P, s);
    const int4 l = P.lf[s].l;
    uint32_t* o = out + 6 * (size_t)r;
    o[0] = s;
    o[1] = (uint32_t)id;
    o[2] = (uint32_t)(id >> 32);
    o[3] = (uint32_t)l.x;
    o[4] = (uint32_t)l.y;
    o[5] = (uint32_t)l.z;
}

// Scatter of live records into a cleared pool; a block or pointer out of
// range raises the pointer flag and is skipped.
__global__ void k_import_live(Pool P, uint32_t n, const uint32_t* in)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* v = in + 6 * (size_t)i;
    const uint32_t s = v[0];
    const int32_t t = (int32_t)v[3], x = (int32_t)v[4], p = (int32_t)v[5];
    const bool ok = s < P.cap && (t == -1 || slot_ok(P, t)) && (x == -1 || slot_ok(P, x)) && (p == -1 || slot_ok(P, p));
    if (!ok) {
        raise_err(P, kErrPointer);
        return;
    }
    P.id[s] = (uint64_t)v[1] | ((uint64_t)v[2] << 32);
    P.lf[s].l = make_int4(t, x, p, 0);
}

// Triangle export: the cached world positions of every live bisector's
// three vertices, in rank order, 9 floats per triangle.  Each workgroup
// stages its 256 triangles in LDS and writes them as one contiguous run.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_export_triangles(Pool P, uint32_t L, float* out)
{
    __shared__ float stage[kBlock * 9];
    const uint32_t r0 = blockIdx.x * kBlock;
    const uint32_t r = r0 + threadIdx.x;
    if (r < L) {
        const T4<R>* w = world_rec<R>(P, P.live[r]);
        const T4<R> a = w[0], b = w[1], c = w[2];
        float* t = stage + 9 * threadIdx.x;
        t[0] = (float)a.x; t[1] = (float)a.y; t[2] = (float)a.z;
        t[3] = (float)b.x; t[4] = (float)b.y; t[5] = (float)b.z;
        t[6] = (float)c.x; t[7] = (float)c.y; t[8] = (float)c.z;
    }
    __syncthreads();
    const uint32_t n = 9u * ((L - r0) < (uint32_t)kBlock ? (L - r0) : (uint32_t)kBlock);
    float* o = out + 9 * (size_t)r0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) o[i] = stage[i];
}

// counters of every instance of a batch, gathered into one array
__global__ void k_gather_counters(Batch B, Counters* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B.n) return;
    out[i] = *B.inst[i].P.ctr;
}

// ---------------------------------------------------------------------------
// host-side launch sequences
// ---------------------------------------------------------------------------

static inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

uint32_t word_groups(const Pool& P) { return cdiv(P.W, kWordsPerBlock); }

int reduce_levels(const Pool& P)
{
    const int LW = word_level(P.D);
    return LW < P.sub ? LW : P.sub;
}

uint32_t reduce_groups(const Pool& P) { return P.W >> reduce_levels(P); }

uint32_t phase_groups_host(const Pool& P, int ph)
{
    switch (ph) {
    case kPhEnum:
    case kPhFree: return word_groups(P);
    case kPhVote:
    case kPhFill: return list_groups(P);
    case kPhClass:
    case kPhBudget:
    case kPhWalk:
    case kPhOwners:
    case kPhResolve: return P.G;
    case kPhRedSub: return reduce_groups(P);
    default: return 1u;
    }
}

uint32_t persist_items_host(uint32_t groups)
{
    const uint32_t sp = (groups + kPersistItems - 1) / kPersistItems;
    return (groups + sp - 1) / sp;
}

size_t workspace_layout(int32_t H, int32_t D, int32_t f64, Pool* P, char* base)
{
    const uint64_t cap = 1ull << D;
    const uint64_t W = cap >= 32 ? cap / 32 : 1;                 // a pool below 32 blocks has one partial word
    const uint64_t TW = 2ull << word_level(D);                   // tree nodes 1 .. 2^(LW+1) - 1
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_id = take(8 * cap), o_lf = take(sizeof(LinkFwd) * cap);
    const size_t vrec = f64 ? 3 * sizeof(double4) : 3 * sizeof(float4);   // one vertex-cache record
    const size_t o_world = take(vrec * cap), o_cmd = take(4 * cap);
    const size_t o_bits = take(4 * W), o_tree = take(4 * TW), o_live = take(4 * cap);
    const size_t o_free = take(4 * cap), o_list = take(8 * cap), o_lpre = take(4 * cap), o_lcnt = take(4 * (size_t)kMaxRankGroups);
    const size_t o_part = take(sizeof(uint2) * kMaxRankGroups), o_ctr = take(sizeof(Counters));
    const size_t o_slane = take(4 * (size_t)kStLanes * kLaneWords);
    const size_t o_root = take((f64 ? 72 : 36) * (size_t)H);
    if (P) {
        P->id = reinterpret_cast<uint64_t*>(base + o_id);
        P->lf = reinterpret_cast<LinkFwd*>(base + o_lf);
        P->vworld = reinterpret_cast<float4*>(base + o_world);
        P->cmd = reinterpret_cast<uint32_t*>(base + o_cmd);
        P->bits = reinterpret_cast<uint32_t*>(base + o_bits);
        P->tree = reinterpret_cast<uint32_t*>(base + o_tree);
        P->live = reinterpret_cast<uint32_t*>(base + o_live);
        P->freel = reinterpret_cast<uint32_t*>(base + o_free);
        P->list = reinterpret_cast<uint2*>(base + o_list);
        P->lpre = reinterpret_cast<uint32_t*>(base + o_lpre);
        P->lcnt = reinterpret_cast<uint32_t*>(base + o_lcnt);
        P->part = reinterpret_cast<uint2*>(base + o_part);
        P->ctr = reinterpret_cast<Counters*>(base + o_ctr);
        P->slane = reinterpret_cast<uint32_t*>(base + o_slane);
        P->root = reinterpret_cast<float*>(base + o_root);
        P->D = D;
        P->H = H;
        P->cap = (uint32_t)cap;
        P->W = (uint32_t)W;
        P->f64 = f64 ? 1 : 0;
    }
    return off;
}

Launch single_launch(const Pool& P, const LodK& K, const uint8_t* inj)
{
    Launch X{};
    X.batched = false;
    X.f64 = P.f64 != 0;
    X.one.P = P;
    X.one.K = K;
    X.one.inj = inj;
    X.B.n = 0;
    X.n_inst = 1;
    X.grid_rank = P.G;
    X.grid_word = word_groups(P);
    X.grid_red = reduce_groups(P);
    X.grid_list = list_groups(P);
    return X;
}

template <bool kB>
static hipError_t reduce_seq(const Launch& X, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_sub<kB>, dim3(X.grid_red), dim3(kBlock), 0, s, X.B, X.one);
    hipLaunchKernelGGL(k_reduce_top<kB>, dim3(X.n_inst), dim3(1024), 0, s, X.B, X.one);
    return hipGetLastError();
}

template <bool kB>
static hipError_t enumerate_seq(const Launch& X, hipStream_t s)
{
    hipLaunchKernelGGL(k_enumerate<kB>, dim3(X.grid_word), dim3(kBlock), 0, s, X.B, X.one);
    return hipGetLastError();
}

template <bool kB, typename R>
static hipError_t frame_seq(const Launch& X, hipStream_t s, const StageEvents* ev)
{
    const dim3 g(X.grid_rank), b(kBlock), gw(X.grid_word), gl(X.grid_list);
    auto mark = [&](int stage, bool begin) {
        if (ev && ev->stage == stage) (void)hipEventRecord(begin ? ev->begin : ev->end, s);
    };
    enum { kEnum = 1, kClass, kVote, kBudget, kChain, kOwners, kOffsets, kFree, kFill, kResolve, kReduce, kFrame };
    mark(kFrame, true);
    mark(kEnum, true);
    hipLaunchKernelGGL(k_enumerate<kB>, gw, b, 0, s, X.B, X.one);
    mark(kEnum, false);
    mark(kClass, true);
    hipLaunchKernelGGL((k_classify<kB, R>), g, b, 0, s, X.B, X.one);
    mark(kClass, false);
    mark(kVote, true);
    hipLaunchKernelGGL(k_vote<kB>, gl, b, 0, s, X.B, X.one);
    mark(kVote, false);
    mark(kBudget, true);
    hipLaunchKernelGGL(k_budget<kB>, g, b, 0, s, X.B, X.one);
    mark(kBudget, false);
    mark(kChain, true);
    hipLaunchKernelGGL(k_walk<kB>, g, b, 0, s, X.B, X.one);
    mark(kChain, false);
    mark(kOwners, true);
    hipLaunchKernelGGL(k_owners<kB>, g, b, 0, s, X.B, X.one);
    mark(kOwners, false);
    mark(kFree, true);
    hipLaunchKernelGGL(k_freelist<kB>, gw, b, 0, s, X.B, X.one);
    mark(kFree, false);
    mark(kFill, true);
    hipLaunchKernelGGL((k_fill<kB, R>), gl, b, 0, s, X.B, X.one);
    mark(kFill, false);
    mark(kResolve, true);
    hipLaunchKernelGGL(k_resolve<kB>, g, b, 0, s, X.B, X.one);
    mark(kResolve, false);
    mark(kReduce, true);
    hipError_t e = reduce_seq<kB>(X, s);
    mark(kReduce, false);
    mark(kFrame, false);
    return e;
}

template <typename R>
static hipError_t persist_seq(const Launch& X, hipStream_t s)
{
    const uint32_t n = X.n_inst * (uint32_t)kPhCount;
    hipLaunchKernelGGL(k_persist_clear, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, X.W, n);
    hipLaunchKernelGGL(k_persist<R>, dim3(X.persist_groups), dim3(kBlock), 0, s, X.B, X.W);
    return hipGetLastError();
}

uint32_t persist_resident_groups(bool f64)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = f64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist<double>, kBlock, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist<float>, kBlock, 0);
    if (e != hipSuccess || per < 1 || cus < 1) return 0;
    return (uint32_t)cus * (uint32_t)per;
}

hipError_t launch_frame(const Launch& X, hipStream_t s, const StageEvents* ev)
{
    if (X.batched && X.persistent) return X.f64 ? persist_seq<double>(X, s) : persist_seq<float>(X, s);
    if (X.f64) return X.batched ? frame_seq<true, double>(X, s, ev) : frame_seq<false, double>(X, s, ev);
    return X.batched ? frame_seq<true, float>(X, s, ev) : frame_seq<false, float>(X, s, ev);
}

hipError_t launch_reduce(const Launch& X, hipStream_t s)
{
    return X.batched ? reduce_seq<true>(X, s) : reduce_seq<false>(X, s);
}

hipError_t launch_enumerate(const Launch& X, hipStream_t s)
{
    return X.batched ? enumerate_seq<true>(X, s) : enumerate_seq<false>(X, s);
}

hipError_t launch_refresh(const Launch& X, hipStream_t s, bool from_ids)
{
    hipError_t e = launch_enumerate(X, s);
    if (e != hipSuccess) return e;
    const dim3 g(X.grid_rank), b(kBlock);
    if (X.f64) {
        if (X.batched) hipLaunchKernelGGL((k_refresh<true, double>), g, b, 0, s, X.B, X.one, from_ids);
        else hipLaunchKernelGGL((k_refresh<false, double>), g, b, 0, s, X.B, X.one, from_ids);
    } else {
        if (X.batched) hipLaunchKernelGGL((k_refresh<true, float>), g, b, 0, s, X.B, X.one, from_ids);
        else hipLaunchKernelGGL((k_refresh<false, float>), g, b, 0, s, X.B, X.one, from_ids);
    }
    return hipGetLastError();
}

hipError_t launch_export_triangles(const Pool& P, uint32_t L, float* out9, hipStream_t s)
{
    if (!L) return hipGetLastError();
    if (P.f64) hipLaunchKernelGGL(k_export_triangles<double>, dim3(cdiv(L, kBlock)), dim3(kBlock), 0, s, P, L, out9);
    else hipLaunchKernelGGL(k_export_triangles<float>, dim3(cdiv(L, kBlock)), dim3(kBlock), 0, s, P, L, out9);
    return hipGetLastError();
}

hipError_t launch_export_live(const Pool& P, uint32_t L, uint32_t* out6, hipStream_t s, bool into_cache)
{
    if (L && into_cache) hipLaunchKernelGGL(k_ids_from_records, dim3(cdiv(L, kBlock)), dim3(kBlock), 0, s, P, L);
    if (L) hipLaunchKernelGGL(k_export_live, dim3(cdiv(L, kBlock)), dim3(kBlock), 0, s, P, L, out6, into_cache);
    return hipGetLastError();
}

hipError_t launch_import_live(const Pool& P, uint32_t n, const uint32_t* in6, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_import_live, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, n, in6);
    return hipGetLastError();
}

hipError_t launch_gather_counters(const Launch& X, Counters* out, hipStream_t s)
{
    if (X.batched && X.n_inst)
        hipLaunchKernelGGL(k_gather_counters, dim3(cdiv(X.n_inst, kBlock)), dim3(kBlock), 0, s, X.B, out);
    return hipGetLastError();
}

hipError_t launch_clear_pool(const Pool& P, hipStream_t s)
{
    const uint32_t blocks = cdiv(P.cap, kBlock) < 4096u ? cdiv(P.cap, kBlock) : 4096u;
    hipLaunchKernelGGL(k_clear_pool, dim3(blocks), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_clear_frame_scratch(const Pool& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_frame_scratch, dim3(1), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_bits_from_ids(const Pool& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_bits_from_ids, dim3(cdiv(P.W, kBlock)), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_gather_ids(const Pool& P, uint32_t r0, uint32_t n, uint64_t* out, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_gather_ids, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, r0, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_canonical(const Pool& P, uint32_t r0, uint32_t n, int32_t* root_h, uint64_t* code,
                                  hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_gather_canonical, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, r0, n, root_h, code);
    return hipGetLastError();
}

hipError_t launch_gather_links(const Pool& P, uint32_t r0, uint32_t n, int32_t* out3, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_gather_links, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, r0, n, out3);
    return hipGetLastError();
}

hipError_t launch_gather_vertices(const Pool& P, uint32_t r0, uint32_t n, float* out9, hipStream_t s)
{
    if (!n) return hipGetLastError();
    const dim3 g(cdiv(n, kBlock)), b(kBlock);
    if (P.f64) hipLaunchKernelGGL((k_gather_vertices<double, float>), g, b, 0, s, P, r0, n, out9);
    else hipLaunchKernelGGL((k_gather_vertices<float, float>), g, b, 0, s, P, r0, n, out9);
    return hipGetLastError();
}

hipError_t launch_gather_vertices64(const Pool& P, uint32_t r0, uint32_t n, double* out9, hipStream_t s)
{
    if (!n) return hipGetLastError();
    const dim3 g(cdiv(n, kBlock)), b(kBlock);
    if (P.f64) hipLaunchKernelGGL((k_gather_vertices<double, double>), g, b, 0, s, P, r0, n, out9);
    else hipLaunchKernelGGL((k_gather_vertices<float, double>), g, b, 0, s, P, r0, n, out9);
    return hipGetLastError();
}

hipError_t launch_gather_decisions(const Pool& P, uint32_t L, uint8_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_bytes, dim3(cdiv(P.cap, kBlock)), dim3(kBlock), 0, s, out, P.cap, (uint8_t)255);
    if (L) hipLaunchKernelGGL(k_gather_decisions, dim3(cdiv(L, kBlock)), dim3(kBlock), 0, s, P, L, out);
    return hipGetLastError();
}

hipError_t launch_export_heap(const Pool& P, uint32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_export_heap, dim3(2048), dim3(kBlock), 0, s, P, out);
    return hipGetLastError();
}

hipError_t launch_export_records(const Pool& P, uint32_t b0, uint32_t n, uint32_t* out5, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_export_records, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, b0, n, out5);
    return hipGetLastError();
}

hipError_t launch_import_records(const Pool& P, uint32_t b0, uint32_t n, const uint32_t* in5, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_import_records, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, b0, n, in5);
    return hipGetLastError();
}

}  // namespace cbtk
