// gfx950 kernels of the per-frame adaptive bisection update.
//
// One frame (Section 3.3 of the paper, nine kernels there) runs here as a
// fixed sequence of launches on one stream, all of them persistent grids
// bounded by device-resident counts (there is no indirect dispatch):
//
//   begin        L = CBT root, F = 2^D - L                   (kernel 1)
//   enumerate    rank -> block list from the bitfield, each
//                workgroup's base taken from the tree       (kernel 2, Alg. 7)
//   classify     decode (Alg. 2), LOD test, merge
//                configuration (Alg. 4); fresh command word  (kernels 3, 4)
//   vote/scan/   merge unanimity; rank-order reservation cut:
//   budget       merges first, then splits of 3d+4 blocks   (kernel 4)
//   chain        split marks along compatibility chains
//                (Alg. 3 as a closure, atomicOr on commands)  (kernel 4)
//   owners/scan  outputs per owner, exclusive offsets        (kernel 5)
//   freelist     first N zero bits of the pre-frame bitfield
//                (Alg. 8 order), bits set                    (kernel 5/8)
//   fill         heap IDs of new bisectors, forwarding table (kernel 6)
//   resolve      neighbour pointers of every new bisector and
//                back-pointers of untouched neighbours
//                (Table 1, Alg. 5, Alg. 6 and compositions)  (kernel 7)
//                consumed bits cleared                       (kernel 8)
//   reduce       sum-reduction tree rebuilt in LDS           (kernel 9)
//
// Determinism: allocation uses scans in rank order instead of an atomic
// counter, every pointer field has exactly one writer, and the only atomics
// are order-free bitwise ORs/ANDs on command words and bitfield words.
//
// Floating point: IEEE binary32, no contraction (built with
// -ffp-contract=off), correctly rounded division and square root.

#include "cbt_internal.h"

#pragma clang fp contract(off)

namespace cbtk {

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

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* sh)
{
    uint32_t t;
    (void)block_excl_scan(v, sh, &t);
    return t;
}

// rank range [r0, r1) of this workgroup: contiguous chunks of ceil(L/G)
__device__ __forceinline__ void rank_range(uint32_t L, uint32_t* r0, uint32_t* r1)
{
    uint32_t chunk = (L + gridDim.x - 1) / gridDim.x;
    uint64_t a = (uint64_t)blockIdx.x * chunk;
    uint64_t b = a + chunk;
    *r0 = (uint32_t)(a < L ? a : L);
    *r1 = (uint32_t)(b < L ? b : L);
}

__device__ __forceinline__ int ilog2_64(uint64_t x) { return 63 - __clzll((long long)x); }

__device__ __forceinline__ void raise_err(const Pool& P, uint32_t e) { atomicOr(&P.ctr->err, e); }

__device__ __forceinline__ uint32_t cmd_of(const int4& l) { return (uint32_t)l.w; }

__device__ __forceinline__ void store_cmd(const Pool& P, uint32_t s, uint32_t cmd)
{
    reinterpret_cast<int*>(&P.link[s])[3] = (int)cmd;
}

__device__ __forceinline__ uint32_t* cmd_ptr(const Pool& P, uint32_t s)
{
    return reinterpret_cast<uint32_t*>(&P.link[s]) + 3;
}

// number of set bits in the words before word w, read off the tree
// (the prefix-sum form of the descent of Alg. 7)
__device__ uint32_t ones_before_word(const Pool& P, uint32_t w)
{
    const int LW = P.D - 5;
    uint32_t node = 1, sum = 0;
    for (int l = LW - 1; l >= 0; --l) {
        uint32_t bit = (w >> l) & 1u;
        if (bit) sum += P.tree[2 * node];
        node = 2 * node + bit;
    }
    return sum;
}

// ---------------------------------------------------------------------------
// kernel: frame begin
// ---------------------------------------------------------------------------

__global__ void k_begin(Pool P)
{
    if (threadIdx.x == 0) {
        uint32_t L = P.tree[1];
        P.ctr->L = L;
        P.ctr->F = P.cap - L;
        P.ctr->Tm = 0;
        P.ctr->Ts = 0;
        P.ctr->N = 0;
    }
    if (threadIdx.x < kStCount) P.ctr->stat[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// kernel: enumerate live blocks (rank order = ascending block index)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_enumerate(Pool P)
{
    __shared__ uint32_t sh[8];
    const uint32_t w0 = blockIdx.x * kWordsPerBlock;
    if (w0 >= P.W) return;
    uint32_t base = ones_before_word(P, w0);
    for (uint32_t it = 0; it < kWordsPerBlock; it += kBlock) {
        const uint32_t w = w0 + it + threadIdx.x;
        uint32_t word = (w < P.W) ? P.bits[w] : 0u;
        uint32_t tot;
        uint32_t o = base + block_excl_scan(__popc(word), sh, &tot);
        while (word) {
            int j = __ffs(word) - 1;
            if (o < P.cap) P.live[o] = w * 32u + (uint32_t)j;
            ++o;
            word &= word - 1;
        }
        base += tot;
    }
}

// ---------------------------------------------------------------------------
// bisector geometry (Eq. 1 / Alg. 2) and the LOD test
// ---------------------------------------------------------------------------

struct V3 {
    float x, y, z;
};

// Splitting matrices applied from the root downwards, one path bit per
// level, most significant first: M0 -> (v0, v2, m), M1 -> (v2, v1, m).
// Scalar registers only (struct selects would be lowered through scratch).
__device__ __forceinline__ void decode(const Pool& P, uint64_t id, int d, V3& A, V3& B, V3& C)
{
    const int64_t h = (int64_t)(id >> d) - ((int64_t)1 << P.k);
    const float* r = P.root + 9 * h;
    float ax = r[0], ay = r[1], az = r[2];
    float bx = r[3], by = r[4], bz = r[5];
    float cx = r[6], cy = r[7], cz = r[8];
    for (int i = d - 1; i >= 0; --i) {
        const bool bit = (id >> i) & 1u;
        const float mx = (ax + bx) * 0.5f, my = (ay + by) * 0.5f, mz = (az + bz) * 0.5f;
        const float nax = bit ? cx : ax, nay = bit ? cy : ay, naz = bit ? cz : az;
        const float nbx = bit ? bx : cx, nby = bit ? by : cy, nbz = bit ? bz : cz;
        ax = nax; ay = nay; az = naz;
        bx = nbx; by = nby; bz = nbz;
        cx = mx; cy = my; cz = mz;
    }
    A = {ax, ay, az};
    B = {bx, by, bz};
    C = {cx, cy, cz};
}

__device__ __forceinline__ float bilinear(const float* T, int res, float s, float t)
{
    float fs = floorf(s), ft = floorf(t);
    const float lim = (float)(res - 2);
    fs = fs < 0.0f ? 0.0f : fs;
    fs = fs > lim ? lim : fs;
    ft = ft < 0.0f ? 0.0f : ft;
    ft = ft > lim ? lim : ft;
    int i0 = (int)fs, j0 = (int)ft;
    i0 = i0 < 0 ? 0 : (i0 > res - 2 ? res - 2 : i0);   // bounds guard (no-op unless NaN)
    j0 = j0 < 0 ? 0 : (j0 > res - 2 ? res - 2 : j0);
    const float fx = s - fs, fy = t - ft;
    const float* r0 = T + (size_t)j0 * res + i0;
    const float* r1 = r0 + res;
    const float a = r0[0], b = r0[1], c = r1[0], e = r1[1];
    const float top = a + fx * (b - a);
    const float bot = c + fx * (e - c);
    return top + fy * (bot - top);
}

__device__ __forceinline__ float sample_cube(const LodK& K, float x, float y, float z)
{
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int f;
    float u, v;
    if (ax >= ay && ax >= az) {
        f = x >= 0.0f ? 0 : 1;
        u = __fdiv_rn(y, ax);
        v = __fdiv_rn(z, ax);
    } else if (ay >= az) {
        f = y >= 0.0f ? 2 : 3;
        u = __fdiv_rn(x, ay);
        v = __fdiv_rn(z, ay);
    } else {
        f = z >= 0.0f ? 4 : 5;
        u = __fdiv_rn(x, az);
        v = __fdiv_rn(y, az);
    }
    const float hr = 0.5f * (float)(K.res - 1);
    return bilinear(K.table + (size_t)f * K.res * K.res, K.res, (u + 1.0f) * hr, (v + 1.0f) * hr);
}

__device__ __forceinline__ V3 world(const LodK& K, V3 v)
{
    if (K.mode == 1) {
        const float len = __builtin_sqrtf((v.x * v.x + v.y * v.y) + v.z * v.z);
        const float nx = __fdiv_rn(v.x, len), ny = __fdiv_rn(v.y, len), nz = __fdiv_rn(v.z, len);
        const float h = sample_cube(K, nx, ny, nz);
        const float sc = 1.0f + K.amp * h;
        return {nx * sc, ny * sc, nz * sc};
    }
    if (K.mode == 2) {
        const float r1 = (float)(K.res - 1);
        const float h = bilinear(K.table, K.res, v.x * r1, v.y * r1);
        return {v.x, v.y, v.z + K.amp * h};
    }
    return v;
}

// Projected base-edge length test without division (see the host-side
// documentation of cbt_lod_params): returns the decision code.
__device__ __forceinline__ uint32_t lod_decide(const LodK& K, V3 a, V3 b, V3 c)
{
    V3 p[3] = {world(K, a), world(K, b), world(K, c)};
    float vx[3], vy[3], vz[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float q0 = p[i].x - K.cam[0], q1 = p[i].y - K.cam[1], q2 = p[i].z - K.cam[2];
        vx[i] = (q0 * K.right[0] + q1 * K.right[1]) + q2 * K.right[2];
        vy[i] = (q0 * K.up[0] + q1 * K.up[1]) + q2 * K.up[2];
        vz[i] = (q0 * K.fwd[0] + q1 * K.fwd[1]) + q2 * K.fwd[2];
    }
    bool on = true, ol = true, orr = true, ob = true, ot = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float zx = K.tx * vz[i], zy = K.ty * vz[i];
        on = on && (vz[i] < K.znear);
        orr = orr && (vx[i] > zx);
        ol = ol && (vx[i] < -zx);
        ot = ot && (vy[i] > zy);
        ob = ob && (vy[i] < -zy);
    }
    if (on || ol || orr || ob || ot) return kMerge;
    if (vz[0] < K.znear || vz[1] < K.znear) return kSplit;
    const float ex = vx[1] * vz[0] - vx[0] * vz[1];
    const float ey = vy[1] * vz[0] - vy[0] * vz[1];
    const float A = K.f2 * (ex * ex + ey * ey);
    const float zz = vz[0] * vz[1];
    const float z4 = zz * zz;
    const float Bs = K.t2s * z4;
    const float Bm = K.t2m * z4;
    if (A > Bs) return kSplit;
    if (A < Bm) return kMerge;
    return kKeep;
}

// ---------------------------------------------------------------------------
// merge configurations (Alg. 4)
// ---------------------------------------------------------------------------

struct Members {
    int n;        // 0, 2 (border pair) or 4 (cycle)
    int32_t m[4]; // j1, j2, j3, j4
};

__device__ __forceinline__ bool slot_ok(const Pool& P, int32_t s) { return (uint32_t)s < P.cap; }

// Alg. 4 from bisector s (depth >= 1) on the pre-frame pointers.
__device__ Members merge_members(const Pool& P, int32_t s, uint64_t id, int4 l1)
{
    Members M;
    M.n = 0;
    const bool bit = id & 1u;
    const int32_t j2 = bit ? l1.z : l1.y;
    const int32_t j3 = bit ? l1.y : l1.z;
    if (j2 < 0) return M;
    if (!slot_ok(P, j2)) { raise_err(P, kErrPointer); return M; }
    const uint64_t id2 = P.id[j2];
    if ((id2 >> 1) != (id >> 1)) return M;
    M.m[0] = s;
    M.m[1] = j2;
    if (j3 < 0) { M.n = 2; return M; }
    if (!slot_ok(P, j3)) { raise_err(P, kErrPointer); return M; }
    const uint64_t id3 = P.id[j3];
    if (ilog2_64(id3) != ilog2_64(id)) return M;
    const int4 l3 = P.link[j3];
    const int32_t j4 = bit ? l3.y : l3.z;
    if (j4 < 0) return M;
    if (!slot_ok(P, j4)) { raise_err(P, kErrPointer); return M; }
    if ((P.id[j4] >> 1) != (id3 >> 1)) return M;
    M.m[2] = j3;
    M.m[3] = j4;
    M.n = 4;
    return M;
}

// ---------------------------------------------------------------------------
// kernel: classify (decision + merge configuration) -> fresh command word
// ---------------------------------------------------------------------------

template <bool kInjected>
__global__ void __launch_bounds__(kBlock) k_classify(Pool P, LodK K, const uint8_t* inj)
{
    __shared__ uint32_t sh[8];
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    const int maxd = 63 - P.k;
    uint32_t nsplit = 0, nmerge = 0;
    for (uint32_t base = r0; base < r1; base += kBlock) {
        const uint32_t r = base + threadIdx.x;
        if (r < r1) {
            const uint32_t s = P.live[r];
            const uint64_t id = P.id[s];
            const int d = ilog2_64(id) - P.k;
            if (id == 0 || d < 0 || d > maxd || (int64_t)(id >> d) - ((int64_t)1 << P.k) >= P.H) {
                raise_err(P, kErrPointer);   // not a bisector of this mesh
                store_cmd(P, s, kKeep);
                continue;
            }
            uint32_t dec;
            if (kInjected) {
                dec = inj[s];
                if (dec > kMerge) {
                    raise_err(P, kErrDecision);
                    dec = kKeep;
                }
            } else {
                V3 a, b, c;
                decode(P, id, d, a, b, c);
                dec = lod_decide(K, a, b, c);
            }
            if (dec == kMerge && d == 0) dec = kKeep;       // roots never merge
            if (dec == kSplit && d + 1 > maxd) dec = kKeep; // index width
            uint32_t cmd = dec | ((uint32_t)d << kDepthShift);
            if (dec == kMerge) {
                const int4 l1 = P.link[s];
                Members M = merge_members(P, (int32_t)s, id, l1);
                if (M.n) {
                    cmd |= kMCfg | (M.n == 4 ? kMQuad : 0u);
                    bool mn = true;
                    for (int i = 1; i < M.n; ++i) mn = mn && (id < P.id[M.m[i]]);
                    if (mn) cmd |= kMMin;
                }
                ++nmerge;
            }
            if (dec == kSplit) ++nsplit;
            store_cmd(P, s, cmd);
        }
    }
    uint32_t a = block_sum(nsplit, sh);
    uint32_t b = block_sum(nmerge, sh);
    if (threadIdx.x == 0) {
        if (a) atomicAdd(&P.ctr->stat[kStSplitReq], a);
        if (b) atomicAdd(&P.ctr->stat[kStMergeReq], b);
    }
}

// ---------------------------------------------------------------------------
// kernels: merge unanimity and the reservation scan
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_vote(Pool P)
{
    __shared__ uint2 sh2[8];
    __shared__ uint32_t sh[8];
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    uint2 acc = make_uint2(0, 0);
    uint32_t ncfg = 0;
    for (uint32_t base = r0; base < r1; base += kBlock) {
        const uint32_t r = base + threadIdx.x;
        uint2 v = make_uint2(0, 0);
        if (r < r1) {
            const uint32_t s = P.live[r];
            const int4 l = P.link[s];
            const uint32_t cmd = cmd_of(l);
            if ((cmd & kDecMask) == kSplit) v.y = 3u * ((cmd & kDepthMask) >> kDepthShift) + 4u;
            if ((cmd & (kMCfg | kMMin)) == (kMCfg | kMMin)) {
                Members M = merge_members(P, (int32_t)s, P.id[s], l);
                bool ok = M.n == ((cmd & kMQuad) ? 4 : 2);
                for (int i = 1; i < M.n && ok; ++i) {
                    const uint32_t c = *cmd_ptr(P, (uint32_t)M.m[i]);
                    ok = (c & (kDecMask | kMCfg | kMQuad)) == (kMerge | kMCfg | (cmd & kMQuad));
                }
                if (ok) {
                    v.x = (uint32_t)(M.n / 2);
                    ++ncfg;
                }
            }
            P.val[r] = v;
        }
        uint2 tot;
        (void)block_incl_scan_sat(v, sh2, &tot);
        acc = sat_add2(acc, tot);
    }
    uint32_t c = block_sum(ncfg, sh);
    if (threadIdx.x == 0) {
        P.part[blockIdx.x] = acc;
        if (c) atomicAdd(&P.ctr->stat[kStMergeCfg], c);
    }
}

// exclusive saturating scan of the per-workgroup partials (one workgroup of
// 1024 threads, kRankGrid / 1024 partials each); mode 0: the totals are the
// reservations, mode 1: the allocations
__global__ void __launch_bounds__(1024) k_scan_parts(Pool P, int mode)
{
    constexpr int E = kRankGrid / 1024;
    __shared__ uint2 sh[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint2 v[E];
    uint2 loc = make_uint2(0, 0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        v[e] = P.part[threadIdx.x * E + e];
        loc = sat_add2(loc, v[e]);
    }
    const uint2 inc = wave_incl_scan_sat(loc);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint2 pre = make_uint2(0, 0), tot = make_uint2(0, 0);
    for (int i = 0; i < 16; ++i) {
        const uint2 t = sh[i];
        if (i < w) pre = sat_add2(pre, t);
        tot = sat_add2(tot, t);
    }
    const uint32_t ex = __shfl_up(inc.x, 1, 64), ey = __shfl_up(inc.y, 1, 64);
    uint2 run = lane ? sat_add2(pre, make_uint2(ex, ey)) : pre;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        P.part[threadIdx.x * E + e] = run;
        run = sat_add2(run, v[e]);
    }
    if (threadIdx.x == 0) {
        if (mode == 0) {
            P.ctr->Tm = tot.x;
            P.ctr->Ts = tot.y;
        } else {
            P.ctr->N = tot.x;
            if (tot.x > P.ctr->F) raise_err(P, kErrAlloc);
        }
    }
}

// Rank-order cut: merge reservation r accepted when the inclusive merge
// prefix fits in F; split reservation r when all merge reservations plus
// the inclusive split prefix fit in F.
__global__ void __launch_bounds__(kBlock) k_budget(Pool P)
{
    __shared__ uint2 sh2[8];
    __shared__ uint32_t sh[8];
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    const uint32_t F = P.ctr->F, Tm = P.ctr->Tm;
    uint2 carry = P.part[blockIdx.x];
    uint32_t nm = 0, ns = 0;
    for (uint32_t base = r0; base < r1; base += kBlock) {
        const uint32_t r = base + threadIdx.x;
        const uint2 v = r < r1 ? P.val[r] : make_uint2(0, 0);
        uint2 tot;
        const uint2 inc = sat_add2(carry, block_incl_scan_sat(v, sh2, &tot));
        if (r < r1 && (v.x | v.y)) {
            const uint32_t s = P.live[r];
            uint32_t add = 0;
            if (v.x && inc.x <= F) { add |= kMAcc; ++nm; }
            if (v.y && sat_add(Tm, inc.y) <= F) { add |= kSAcc; ++ns; }
            if (add) store_cmd(P, s, *cmd_ptr(P, s) | add);
        }
        carry = sat_add2(carry, tot);
    }
    uint32_t a = block_sum(nm, sh);
    uint32_t b = block_sum(ns, sh);
    if (threadIdx.x == 0) {
        if (a) atomicAdd(&P.ctr->stat[kStMergeAcc], a);
        if (b) atomicAdd(&P.ctr->stat[kStSplitAcc], b);
    }
}

// ---------------------------------------------------------------------------
// kernel: compatibility chains (Alg. 3) as split marks
// ---------------------------------------------------------------------------

// Walk from an accepted initiator through Twin: a same-level twin pair ends
// the chain; a coarser twin receives the mark of the edge it shares (Next or
// Prev) plus its own base mark and the walk continues from it.  A walk stops
// as soon as it finds a base mark already set: whoever set it walks (or
// walked) the same remaining chain, which depends on pre-frame pointers only.
__global__ void __launch_bounds__(kBlock) k_chain(Pool P)
{
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const uint32_t s = P.live[r];
        if (!(*cmd_ptr(P, s) & kSAcc)) continue;
        uint32_t old = atomicOr(cmd_ptr(P, s), kMarkB);
        if (old & kMarkB) continue;
        int32_t cur = (int32_t)s;
        int it = 0;
        for (; it < 130; ++it) {
            const int32_t n = P.link[cur].x;
            if (n < 0) break;
            if (!slot_ok(P, n)) { raise_err(P, kErrPointer); break; }
            const int4 ln = P.link[n];
            if (ln.x == cur) {
                atomicOr(cmd_ptr(P, (uint32_t)n), kMarkB);
                break;
            }
            uint32_t e;
            if (ln.y == cur) e = kMarkN;
            else if (ln.z == cur) e = kMarkP;
            else { raise_err(P, kErrPointer); break; }
            old = atomicOr(cmd_ptr(P, (uint32_t)n), e | kMarkB);
            if (old & kMarkB) break;
            cur = n;
        }
        if (it >= 130) raise_err(P, kErrChain);
    }
}

// ---------------------------------------------------------------------------
// kernels: owners and their allocation offsets
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t split_outputs(uint32_t cmd)
{
    return 2u + ((cmd & kMarkN) ? 1u : 0u) + ((cmd & kMarkP) ? 1u : 0u);
}

__global__ void __launch_bounds__(kBlock) k_owners(Pool P)
{
    __shared__ uint32_t sh[8];
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    uint32_t acc = 0, nexec = 0, nsc = 0, nfree = 0;
    for (uint32_t base = r0; base < r1; base += kBlock) {
        const uint32_t r = base + threadIdx.x;
        uint32_t n = 0;
        if (r < r1) {
            const uint32_t s = P.live[r];
            const int4 l = P.link[s];
            const uint32_t cmd = cmd_of(l);
            if (cmd & kMarks) {
                n = split_outputs(cmd);
                ++nsc;
                ++nfree;
            } else if (cmd & kMAcc) {
                Members M = merge_members(P, (int32_t)s, P.id[s], l);
                bool clean = M.n > 0;
                for (int i = 0; i < M.n; ++i) clean = clean && !(*cmd_ptr(P, (uint32_t)M.m[i]) & kMarks);
                if (clean) {
                    n = (uint32_t)(M.n / 2);
                    for (int i = 0; i < M.n; ++i) atomicOr(cmd_ptr(P, (uint32_t)M.m[i]), kMExec);
                    ++nexec;
                    nfree += (uint32_t)M.n;
                }
            }
            P.val[r].x = n;
        }
        uint32_t tot;
        (void)block_excl_scan(n, sh, &tot);
        acc += tot;
    }
    const uint32_t a = block_sum(nexec, sh);
    const uint32_t b = block_sum(nsc, sh);
    const uint32_t c = block_sum(nfree, sh);
    if (threadIdx.x == 0) {
        P.part[blockIdx.x] = make_uint2(acc, 0);
        if (a) atomicAdd(&P.ctr->stat[kStMergeExec], a);
        if (b) atomicAdd(&P.ctr->stat[kStSplitConsumed], b);
        if (c) atomicAdd(&P.ctr->stat[kStFrees], c);
    }
}

__global__ void __launch_bounds__(kBlock) k_offsets(Pool P)
{
    __shared__ uint32_t sh[8];
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    uint32_t carry = P.part[blockIdx.x].x;
    for (uint32_t base = r0; base < r1; base += kBlock) {
        const uint32_t r = base + threadIdx.x;
        const uint32_t n = r < r1 ? P.val[r].x : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(n, sh, &tot);
        if (r < r1) P.pre[r] = carry + ex;
        carry += tot;
    }
}

// ---------------------------------------------------------------------------
// kernel: the first N free blocks (ZeroToBitID(0..N-1) of the pre-frame
// tree, Alg. 8), marked occupied
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_freelist(Pool P)
{
    __shared__ uint32_t sh[8];
    const uint32_t N = P.ctr->N;
    const uint32_t w0 = blockIdx.x * kWordsPerBlock;
    if (w0 >= P.W || N == 0) return;
    uint32_t zb = 32u * w0 - ones_before_word(P, w0);
    if (zb >= N) return;
    for (uint32_t it = 0; it < kWordsPerBlock; it += kBlock) {
        const uint32_t w = w0 + it + threadIdx.x;
        const uint32_t word = (w < P.W) ? P.bits[w] : 0xffffffffu;
        uint32_t tot;
        uint32_t o = zb + block_excl_scan(__popc(~word), sh, &tot);
        if (w < P.W && o < N) {
            uint32_t inv = ~word, nw = word;
            while (inv && o < N) {
                const int j = __ffs(inv) - 1;
                P.freel[o++] = w * 32u + (uint32_t)j;
                nw |= 1u << j;
                inv &= inv - 1;
            }
            P.bits[w] = nw;
        }
        zb += tot;
        if (zb >= N) break;
    }
}

// ---------------------------------------------------------------------------
// split outputs: roles and heap IDs
// ---------------------------------------------------------------------------

// Forwarding record of a split bisector, by role:
//   0: first child (2x), or its first child (4x) when the Prev edge splits
//   1: second child of the first child (4x+1), Prev edge split only
//   2: second child (2x+1), or its first child (4x+2) when the Next edge splits
//   3: second child of the second child (4x+3), Next edge split only
// Outputs take their blocks in ascending heap-ID order.
__device__ __forceinline__ uint32_t comp(uint4 v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// the two sibling pairs of a merge configuration, even member first
__device__ __forceinline__ void merge_pairs(const Pool& P, const Members& M, int32_t* a0, int32_t* a1,
                                            int32_t* b0, int32_t* b1)
{
    const bool odd = P.id[M.m[0]] & 1u;
    *a0 = odd ? M.m[1] : M.m[0];
    *a1 = odd ? M.m[0] : M.m[1];
    if (M.n == 4) {
        const bool odd3 = P.id[M.m[2]] & 1u;
        *b0 = odd3 ? M.m[3] : M.m[2];
        *b1 = odd3 ? M.m[2] : M.m[3];
    } else {
        *b0 = *b1 = -1;
    }
}

// ---------------------------------------------------------------------------
// kernel: fill new blocks (heap IDs) and the forwarding records
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_fill(Pool P)
{
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    const uint32_t N = P.ctr->N;
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const uint32_t s = P.live[r];
        const int4 l = P.link[s];
        const uint32_t cmd = cmd_of(l);
        const uint32_t base = P.pre[r];
        if (cmd & kMarks) {
            // outputs in ascending heap-ID order take blocks base, base+1, ...
            const bool hn = cmd & kMarkN, hp = cmd & kMarkP;
            const uint32_t cnt = 2u + (hn ? 1u : 0u) + (hp ? 1u : 0u);
            if (base + cnt > N) { raise_err(P, kErrAlloc); continue; }
            const uint32_t q0 = P.freel[base], q1 = P.freel[base + 1];
            const uint32_t q2 = cnt > 2 ? P.freel[base + 2] : 0u, q3 = cnt > 3 ? P.freel[base + 3] : 0u;
            if (q0 >= P.cap || q1 >= P.cap || q2 >= P.cap || q3 >= P.cap) { raise_err(P, kErrAlloc); continue; }
            const uint64_t x = P.id[s];
            uint4 f;
            if (!hn && !hp) {          // 2x, 2x+1
                P.id[q0] = 2 * x;
                P.id[q1] = 2 * x + 1;
                f = make_uint4(q0, 0xffffffffu, q1, 0xffffffffu);
            } else if (hn && !hp) {    // 2x, 4x+2, 4x+3
                P.id[q0] = 2 * x;
                P.id[q1] = 4 * x + 2;
                P.id[q2] = 4 * x + 3;
                f = make_uint4(q0, 0xffffffffu, q1, q2);
            } else if (!hn && hp) {    // 2x+1, 4x, 4x+1
                P.id[q0] = 2 * x + 1;
                P.id[q1] = 4 * x;
                P.id[q2] = 4 * x + 1;
                f = make_uint4(q1, q2, q0, 0xffffffffu);
            } else {                   // 4x, 4x+1, 4x+2, 4x+3
                P.id[q0] = 4 * x;
                P.id[q1] = 4 * x + 1;
                P.id[q2] = 4 * x + 2;
                P.id[q3] = 4 * x + 3;
                f = make_uint4(q0, q1, q2, q3);
            }
            P.fwd[s] = f;
        } else if ((cmd & (kMExec | kMMin)) == (kMExec | kMMin)) {
            const Members M = merge_members(P, (int32_t)s, P.id[s], l);
            if (M.n == 0) { raise_err(P, kErrPointer); continue; }
            int32_t a0, a1, b0, b1;
            merge_pairs(P, M, &a0, &a1, &b0, &b1);
            const uint64_t pa = P.id[a0] >> 1;
            const uint64_t pb = M.n == 4 ? (P.id[b0] >> 1) : 0;
            if (base + (M.n / 2) > N) { raise_err(P, kErrAlloc); continue; }
            uint32_t qa, qb = 0xffffffffu;
            if (M.n == 4) {
                const uint32_t q0 = P.freel[base], q1 = P.freel[base + 1];
                qa = pa < pb ? q0 : q1;
                qb = pa < pb ? q1 : q0;
            } else {
                qa = P.freel[base];
            }
            if (qa >= P.cap || (M.n == 4 && qb >= P.cap)) { raise_err(P, kErrAlloc); continue; }
            P.id[qa] = pa;
            P.fwd[a0] = make_uint4(qa, 0, 0, 0);
            P.fwd[a1] = make_uint4(qa, 0, 0, 0);
            if (M.n == 4) {
                P.id[qb] = pb;
                P.fwd[b0] = make_uint4(qb, 0, 0, 0);
                P.fwd[b1] = make_uint4(qb, 0, 0, 0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// kernel: neighbour pointers (Table 1, Alg. 5/6 and their compositions)
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

__device__ __forceinline__ int32_t link_field(const int4& l, int e) { return e == 0 ? l.x : (e == 1 ? l.y : l.z); }

// New neighbour across (a piece of) edge e of the consumed bisector b, seen
// from its output x.  The old neighbour n is found through b's pre-frame
// pointer; n is then untouched (x takes n, and n's back-pointer is
// rewritten to x -- its only writer), split (the output of n covering the
// same piece: on a shared edge the halves swap between bisectors of equal
// depth and keep their names across a depth difference of one), or merged
// (its parent).
__device__ int32_t resolve_edge(const Pool& P, int32_t b, const int4& lb, int db, int e, int piece, uint32_t x)
{
    const int32_t n = link_field(lb, e);
    if (n < 0) return -1;
    if (!slot_ok(P, n)) { raise_err(P, kErrPointer); return -1; }
    const int4 ln = P.link[n];
    const int f = ln.x == b ? 0 : (ln.y == b ? 1 : (ln.z == b ? 2 : -1));
    if (f < 0) { raise_err(P, kErrPointer); return -1; }
    const uint32_t cn = cmd_of(ln);
    if (cn & kMarks) {
        const int dn = (int)((cn & kDepthMask) >> kDepthShift);
        int pn = piece;
        if (piece != kWhole && dn == db) pn = piece == kHalf0 ? kHalf1 : kHalf0;
        const int role = cover_role(cn & kMarks, f, pn);
        if (role < 0) { raise_err(P, kErrEdge); return -1; }
        return (int32_t)comp(P.fwd[n], role);
    }
    if (cn & kMExec) return (int32_t)P.fwd[n].x;
    if (piece != kWhole) { raise_err(P, kErrEdge); return -1; }
    reinterpret_cast<int*>(&P.link[n])[f] = (int)x;
    return n;
}

__device__ __forceinline__ void store_link(const Pool& P, uint32_t q, int32_t t, int32_t n, int32_t p)
{
    if (q < P.cap) P.link[q] = make_int4(t, n, p, 0);
    else raise_err(P, kErrAlloc);
}

__device__ __forceinline__ void clear_bit(const Pool& P, uint32_t s)
{
    atomicAnd(&P.bits[s >> 5], ~(1u << (s & 31u)));
}

__global__ void __launch_bounds__(kBlock) k_resolve(Pool P)
{
    uint32_t r0, r1;
    rank_range(P.ctr->L, &r0, &r1);
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += kBlock) {
        const int32_t b = (int32_t)P.live[r];
        const int4 lb = P.link[b];
        const uint32_t cmd = cmd_of(lb);
        if (cmd & kMarks) {
            const int db = (int)((cmd & kDepthMask) >> kDepthShift);
            const bool hn = cmd & kMarkN, hp = cmd & kMarkP;
            const uint4 f = P.fwd[b];
            if (!hp) {  // first child (v0, v2, m)
                store_link(P, f.x, resolve_edge(P, b, lb, db, kEdgeP, kWhole, f.x), (int32_t)f.z,
                           resolve_edge(P, b, lb, db, kEdgeT, kHalf0, f.x));
            } else {    // its two children
                store_link(P, f.x, resolve_edge(P, b, lb, db, kEdgeT, kHalf0, f.x), (int32_t)f.y,
                           resolve_edge(P, b, lb, db, kEdgeP, kHalf1, f.x));
                store_link(P, f.y, (int32_t)f.z, resolve_edge(P, b, lb, db, kEdgeP, kHalf0, f.y), (int32_t)f.x);
            }
            if (!hn) {  // second child (v2, v1, m)
                store_link(P, f.z, resolve_edge(P, b, lb, db, kEdgeN, kWhole, f.z),
                           resolve_edge(P, b, lb, db, kEdgeT, kHalf1, f.z), (int32_t)(hp ? f.y : f.x));
            } else {    // its two children
                store_link(P, f.z, (int32_t)(hp ? f.y : f.x), (int32_t)f.w,
                           resolve_edge(P, b, lb, db, kEdgeN, kHalf1, f.z));
                store_link(P, f.w, resolve_edge(P, b, lb, db, kEdgeT, kHalf1, f.w),
                           resolve_edge(P, b, lb, db, kEdgeN, kHalf0, f.w), (int32_t)f.z);
            }
            clear_bit(P, (uint32_t)b);
        } else if ((cmd & (kMExec | kMMin)) == (kMExec | kMMin)) {
            const Members M = merge_members(P, b, P.id[b], lb);
            if (M.n == 0) { raise_err(P, kErrPointer); continue; }
            int32_t a0, a1, b0, b1;
            merge_pairs(P, M, &a0, &a1, &b0, &b1);
            const uint32_t qa = P.fwd[a0].x;
            const uint32_t qb = M.n == 4 ? P.fwd[b0].x : 0xffffffffu;
            // parent of a sibling pair: Next edge = odd child's base edge,
            // Prev edge = even child's base edge, Twin = the other parent
            {
                const int4 l0 = P.link[a0], l1 = P.link[a1];
                const int d0 = (int)((cmd_of(l0) & kDepthMask) >> kDepthShift);
                const int32_t nn = resolve_edge(P, a1, l1, d0, kEdgeT, kWhole, qa);
                const int32_t pp = resolve_edge(P, a0, l0, d0, kEdgeT, kWhole, qa);
                store_link(P, qa, M.n == 4 ? (int32_t)qb : -1, nn, pp);
            }
            if (M.n == 4) {
                const int4 l0 = P.link[b0], l1 = P.link[b1];
                const int d0 = (int)((cmd_of(l0) & kDepthMask) >> kDepthShift);
                const int32_t nn = resolve_edge(P, b1, l1, d0, kEdgeT, kWhole, qb);
                const int32_t pp = resolve_edge(P, b0, l0, d0, kEdgeT, kWhole, qb);
                store_link(P, qb, (int32_t)qa, nn, pp);
            }
            for (int i = 0; i < M.n; ++i) clear_bit(P, (uint32_t)M.m[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// kernels: sum-reduction tree (down to the word level; the levels below a
// word are popcounts of the bitfield and are never stored)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_reduce_sub(Pool P)
{
    __shared__ uint32_t buf[2][1 << kReduceSub];
    const int LW = P.D - 5;
    const int SUB = LW < kReduceSub ? LW : kReduceSub;
    const uint32_t wpb = 1u << SUB;
    const uint32_t w0 = blockIdx.x * wpb;
    for (uint32_t i = threadIdx.x; i < wpb; i += kBlock) {
        const uint32_t c = __popc(P.bits[w0 + i]);
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
            P.tree[(1u << (LW - lvl)) + (blockIdx.x << (SUB - lvl)) + i] = v;
        }
        __syncthreads();
        src ^= 1;
    }
}

__global__ void __launch_bounds__(1024) k_reduce_top(Pool P)
{
    const int LW = P.D - 5;
    const int top = LW - kReduceSub;   // levels [0, top) remain
    for (int lvl = top - 1; lvl >= 0; --lvl) {
        const uint32_t n = 1u << lvl;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t node = n + i;
            P.tree[node] = P.tree[2 * node] + P.tree[2 * node + 1];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// kernels used by queries and restore
// ---------------------------------------------------------------------------

__global__ void k_bits_from_ids(Pool P)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= P.W) return;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j)
        if (P.id[w * 32u + j] != 0) word |= 1u << j;
    P.bits[w] = word;
}

__global__ void k_gather_ids(Pool P, uint32_t r0, uint32_t n, uint64_t* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = P.id[P.live[r0 + i]];
}

__global__ void k_gather_links(Pool P, uint32_t r0, uint32_t n, int32_t* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 l = P.link[P.live[r0 + i]];
    out[3 * (size_t)i + 0] = l.x;
    out[3 * (size_t)i + 1] = l.y;
    out[3 * (size_t)i + 2] = l.z;
}

__global__ void k_gather_vertices(Pool P, uint32_t r0, uint32_t n, float* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t id = P.id[P.live[r0 + i]];
    const int d = ilog2_64(id) - P.k;
    V3 a = {0, 0, 0}, b = a, c = a;
    if (id != 0 && d >= 0 && d <= 63 - P.k && (int64_t)(id >> d) - ((int64_t)1 << P.k) < P.H)
        decode(P, id, d, a, b, c);
    float* o = out + 9 * (size_t)i;
    o[0] = a.x; o[1] = a.y; o[2] = a.z;
    o[3] = b.x; o[4] = b.y; o[5] = b.z;
    o[6] = c.x; o[7] = c.y; o[8] = c.z;
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
    out[s] = (uint8_t)(*cmd_ptr(P, s) & kDecMask);
}

__global__ void k_export_heap(Pool P, uint32_t* out)
{
    const uint64_t total = 2ull * P.cap;
    const int LW = P.D - 5;
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

// ---------------------------------------------------------------------------
// host-side launch sequences
// ---------------------------------------------------------------------------

static inline uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

size_t workspace_layout(int32_t H, int32_t D, Pool* P, char* base)
{
    const uint64_t cap = 1ull << D;
    const uint64_t W = cap / 32;
    const uint64_t TW = 1ull << (D - 4);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_id = take(8 * cap), o_link = take(16 * cap), o_fwd = take(16 * cap);
    const size_t o_bits = take(4 * W), o_tree = take(4 * TW), o_live = take(4 * cap);
    const size_t o_val = take(8 * cap), o_pre = take(4 * cap), o_free = take(4 * cap);
    const size_t o_part = take(sizeof(uint2) * kRankGrid), o_ctr = take(sizeof(Counters));
    const size_t o_root = take(36 * (size_t)H);
    if (P) {
        P->id = reinterpret_cast<uint64_t*>(base + o_id);
        P->link = reinterpret_cast<int4*>(base + o_link);
        P->fwd = reinterpret_cast<uint4*>(base + o_fwd);
        P->bits = reinterpret_cast<uint32_t*>(base + o_bits);
        P->tree = reinterpret_cast<uint32_t*>(base + o_tree);
        P->live = reinterpret_cast<uint32_t*>(base + o_live);
        P->val = reinterpret_cast<uint2*>(base + o_val);
        P->pre = reinterpret_cast<uint32_t*>(base + o_pre);
        P->freel = reinterpret_cast<uint32_t*>(base + o_free);
        P->part = reinterpret_cast<uint2*>(base + o_part);
        P->ctr = reinterpret_cast<Counters*>(base + o_ctr);
        P->root = reinterpret_cast<float*>(base + o_root);
        P->D = D;
        P->H = H;
        P->cap = (uint32_t)cap;
        P->W = (uint32_t)W;
    }
    return off;
}

hipError_t launch_reduce(const Pool& P, hipStream_t s)
{
    const int LW = P.D - 5;
    const int SUB = LW < kReduceSub ? LW : kReduceSub;
    const uint32_t blocks = P.W >> SUB;
    hipLaunchKernelGGL(k_reduce_sub, dim3(blocks), dim3(kBlock), 0, s, P);
    if (LW > kReduceSub) hipLaunchKernelGGL(k_reduce_top, dim3(1), dim3(1024), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_enumerate(const Pool& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, P);
    hipLaunchKernelGGL(k_enumerate, dim3(cdiv(P.W, kWordsPerBlock)), dim3(kBlock), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_frame(const Pool& P, const LodK& K, const uint8_t* decisions, hipStream_t s,
                        const StageEvents* ev)
{
    const dim3 g(kRankGrid), b(kBlock);
    const dim3 gw(cdiv(P.W, kWordsPerBlock));
    auto mark = [&](int stage, bool begin) {
        if (ev && ev->stage == stage) (void)hipEventRecord(begin ? ev->begin : ev->end, s);
    };
    enum { kEnum = 1, kClass, kVote, kBudget, kChain, kOwners, kOffsets, kFree, kFill, kResolve, kReduce, kFrame };
    mark(kFrame, true);
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, P);
    mark(kEnum, true);
    hipLaunchKernelGGL(k_enumerate, gw, b, 0, s, P);
    mark(kEnum, false);
    mark(kClass, true);
    if (decisions) hipLaunchKernelGGL(k_classify<true>, g, b, 0, s, P, K, decisions);
    else hipLaunchKernelGGL(k_classify<false>, g, b, 0, s, P, K, decisions);
    mark(kClass, false);
    mark(kVote, true);
    hipLaunchKernelGGL(k_vote, g, b, 0, s, P);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, P, 0);
    mark(kVote, false);
    mark(kBudget, true);
    hipLaunchKernelGGL(k_budget, g, b, 0, s, P);
    mark(kBudget, false);
    mark(kChain, true);
    hipLaunchKernelGGL(k_chain, g, b, 0, s, P);
    mark(kChain, false);
    mark(kOwners, true);
    hipLaunchKernelGGL(k_owners, g, b, 0, s, P);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, P, 1);
    mark(kOwners, false);
    mark(kOffsets, true);
    hipLaunchKernelGGL(k_offsets, g, b, 0, s, P);
    mark(kOffsets, false);
    mark(kFree, true);
    hipLaunchKernelGGL(k_freelist, gw, b, 0, s, P);
    mark(kFree, false);
    mark(kFill, true);
    hipLaunchKernelGGL(k_fill, g, b, 0, s, P);
    mark(kFill, false);
    mark(kResolve, true);
    hipLaunchKernelGGL(k_resolve, g, b, 0, s, P);
    mark(kResolve, false);
    mark(kReduce, true);
    hipError_t e = launch_reduce(P, s);
    mark(kReduce, false);
    mark(kFrame, false);
    return e;
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

hipError_t launch_gather_links(const Pool& P, uint32_t r0, uint32_t n, int32_t* out3, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_gather_links, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, r0, n, out3);
    return hipGetLastError();
}

hipError_t launch_gather_vertices(const Pool& P, uint32_t r0, uint32_t n, float* out9, hipStream_t s)
{
    if (n) hipLaunchKernelGGL(k_gather_vertices, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, P, r0, n, out9);
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

}  // namespace cbtk
