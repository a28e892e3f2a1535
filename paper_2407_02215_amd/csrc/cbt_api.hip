// Host side of the C ABI declared in include/cbt.h: argument and mesh
// validation, root bisectors (Section 2.2, Alg. 1), workspace carving, frame
// constants, and the query / snapshot paths.  All device work is done by the
// kernels of cbt_kernels.hip on the caller's stream.

#include "cbt_host.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

using cbtk::Counters;
using cbtk::LodK;
using cbtk::Pool;

static constexpr int kMaxTimed = 8192;

static thread_local char g_err[512] = "";

namespace cbth {

cbt_status fail(cbt_handle h, cbt_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_err, buf, sizeof buf);
    if (h) std::memcpy(h->err, buf, sizeof buf);
    return st;
}

// Pinned counter mirrors come from slabs of 4096 slots allocated once and
// kept for the life of the process: pinned allocations are slow and may
// synchronise the device, which would stall servers that admit and evict
// instances all the time.
namespace {
std::mutex g_pin_mu;
std::vector<Counters*> g_pin_free;
}  // namespace

Counters* pinned_counters()
{
    std::lock_guard<std::mutex> lock(g_pin_mu);
    if (g_pin_free.empty()) {
        constexpr size_t kSlots = 4096;
        Counters* slab = nullptr;
        if (hipHostMalloc(reinterpret_cast<void**>(&slab), sizeof(Counters) * kSlots, hipHostMallocDefault) !=
            hipSuccess)
            return nullptr;
        for (size_t i = kSlots; i-- > 0;) g_pin_free.push_back(slab + i);
    }
    Counters* c = g_pin_free.back();
    g_pin_free.pop_back();
    return c;
}

void release_counters(Counters* c)
{
    if (!c) return;
    std::lock_guard<std::mutex> lock(g_pin_mu);
    g_pin_free.push_back(c);
}

cbt_status hip_fail(cbt_handle h, hipError_t e, const char* what)
{
    if (h) h->failed = 1;
    return fail(h, CBT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Frame constants in double precision.  Binary32 instances round each of
// them once to float on the device; binary64 instances use them as is.
void make_lodk(const cbt_camera* c, const cbt_lod_params* lp, LodK* K)
{
    const double f[3] = {c->fwd[0], c->fwd[1], c->fwd[2]};
    const double u[3] = {c->up[0], c->up[1], c->up[2]};
    const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const double fw[3] = {f[0] / fl, f[1] / fl, f[2] / fl};
    double r[3] = {fw[1] * u[2] - fw[2] * u[1], fw[2] * u[0] - fw[0] * u[2], fw[0] * u[1] - fw[1] * u[0]};
    const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    r[0] /= rl;
    r[1] /= rl;
    r[2] /= rl;
    const double up[3] = {r[1] * fw[2] - r[2] * fw[1], r[2] * fw[0] - r[0] * fw[2], r[0] * fw[1] - r[1] * fw[0]};
    const double th = std::tan(0.5 * (double)c->fovy);
    const double focal = 0.5 * (double)c->height / th;
    for (int i = 0; i < 3; ++i) {
        K->cam[i] = c->pos[i];
        K->right[i] = r[i];
        K->up[i] = up[i];
        K->fwd[i] = fw[i];
    }
    K->f2 = focal * focal;
    if (lp->criterion == CBT_CRIT_AREA) {   // twice the target areas
        K->t2s = 2.0 * (double)lp->split_px;
        K->t2m = 2.0 * (double)lp->merge_px;
    } else {                                // squared target lengths
        K->t2s = (double)lp->split_px * (double)lp->split_px;
        K->t2m = (double)lp->merge_px * (double)lp->merge_px;
    }
    K->crit = lp->criterion;
    K->tx = th * (double)c->width / (double)c->height;
    K->ty = th;
    K->znear = c->znear;
    K->table = lp->table;
    K->res = lp->table_res;
    K->amp = lp->amplitude;
    K->mode = lp->mode;
}

cbt_status check_lod(cbt_handle h, const cbt_camera* c, const cbt_lod_params* lp)
{
    if (!c || !lp) return fail(h, CBT_E_ARG, "camera and LOD parameters are required");
    if (lp->mode < CBT_MODE_FLAT || lp->mode > CBT_MODE_HEIGHTFIELD) return fail(h, CBT_E_ARG, "unknown LOD mode %d", lp->mode);
    if (lp->criterion != CBT_CRIT_EDGE && lp->criterion != CBT_CRIT_AREA && lp->criterion != CBT_CRIT_DISTANCE)
        return fail(h, CBT_E_ARG, "unknown size criterion %d", lp->criterion);
    if (lp->mode != CBT_MODE_FLAT && (!lp->table || lp->table_res < 2))
        return fail(h, CBT_E_ARG, "LOD mode %d needs a device table of resolution >= 2", lp->mode);
    if (c->width <= 0 || c->height <= 0 || !(c->fovy > 0.0f && c->fovy < 3.14159f))
        return fail(h, CBT_E_ARG, "invalid viewport or field of view");
    return CBT_OK;
}

bool world_changed(const LodK& a, const LodK& b)
{
    return a.mode != b.mode || a.table != b.table || a.res != b.res || a.amp != b.amp;
}

cbt_status stats_from_counters(cbt_handle h, const Counters& c, cbt_frame_stats* stats)
{
    if (c.err) {
        h->failed = 1;
        return fail(h, CBT_E_DEVICE, "device check failed (flags 0x%x)", c.err);
    }
    if (!stats) return CBT_OK;
    std::memset(stats, 0, sizeof *stats);
    stats->live_before = c.L;
    stats->free_before = c.F;
    stats->split_requests = c.stat[cbtk::kStSplitReq];
    stats->split_accepted = c.stat[cbtk::kStSplitAcc];
    stats->merge_requests = c.stat[cbtk::kStMergeReq];
    stats->merge_configs = c.stat[cbtk::kStMergeCfg];
    stats->merge_accepted = c.stat[cbtk::kStMergeAcc];
    stats->merges_executed = c.stat[cbtk::kStMergeExec];
    stats->split_consumed = c.stat[cbtk::kStSplitConsumed];
    stats->allocations = c.N;
    stats->frees = c.stat[cbtk::kStFrees];
    stats->live_after = (int64_t)c.L + c.N - c.stat[cbtk::kStFrees];
    stats->merge_candidates = c.stat[cbtk::kStMergeCand];
    return CBT_OK;
}

// Default schedule: about 512 pool blocks per rank workgroup, within the
// grid limits.
uint32_t default_rank_groups(int32_t D)
{
    const uint64_t g = (1ull << D) / 512;
    return (uint32_t)(g < cbtk::kMinRankGroups ? cbtk::kMinRankGroups
                                               : (g > cbtk::kMaxRankGroups ? cbtk::kMaxRankGroups : g));
}

}  // namespace cbth

using cbth::fail;
using cbth::hip_fail;

static int ceil_log2(int64_t n)
{
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    return k;
}

// Section 2.1 halfedge requirements (see cbt_mesh in cbt.h).
cbt_status cbth::validate_mesh(const cbt_mesh* m)
{
    if (!m || !m->twin || !m->next || !m->prev || !m->vert || !m->pos)
        return fail(nullptr, CBT_E_ARG, "mesh arrays must not be NULL");
    const int32_t H = m->H;
    if (H < 3) return fail(nullptr, CBT_E_MESH, "mesh has %d halfedges, needs >= 3", H);
    if (m->V < 1) return fail(nullptr, CBT_E_MESH, "mesh has no vertices");
    for (int32_t h = 0; h < H; ++h) {
        const int32_t n = m->next[h], p = m->prev[h], t = m->twin[h], v = m->vert[h];
        if (n < 0 || n >= H || p < 0 || p >= H) return fail(nullptr, CBT_E_MESH, "halfedge %d: next/prev out of range", h);
        if (m->prev[n] != h || m->next[p] != h) return fail(nullptr, CBT_E_MESH, "halfedge %d: next/prev not inverse", h);
        if (v < 0 || v >= m->V) return fail(nullptr, CBT_E_MESH, "halfedge %d: vertex out of range", h);
        if (t < -1 || t >= H || t == h) return fail(nullptr, CBT_E_MESH, "halfedge %d: twin out of range", h);
        if (t >= 0) {
            if (m->twin[t] != h) return fail(nullptr, CBT_E_MESH, "halfedge %d: twin not an involution", h);
            if (m->vert[t] != m->vert[n] || m->vert[m->next[t]] != v)
                return fail(nullptr, CBT_E_MESH, "halfedge %d: twin not opposite", h);
            if (t == n || t == p) return fail(nullptr, CBT_E_MESH, "halfedge %d: twin in its own corner", h);
        }
    }
    // face cycles of length >= 3 (visit each cycle once)
    std::vector<uint8_t> seen(H, 0);
    for (int32_t h = 0; h < H; ++h) {
        if (seen[h]) continue;
        int32_t len = 0, g = h;
        do {
            seen[g] = 1;
            g = m->next[g];
            if (++len > H) return fail(nullptr, CBT_E_MESH, "face of halfedge %d does not close", h);
        } while (g != h);
        if (len < 3) return fail(nullptr, CBT_E_MESH, "face of halfedge %d has %d sides", h, len);
    }
    return CBT_OK;
}

// Alg. 1 per root: v0 = Vert(h), v1 = Vert(Next(h)), v2 = mean of the face's
// vertices.  The mean is accumulated once per face, from the face's smallest
// halfedge index along Next, in binary32, then divided by the side count, so
// every root of a face shares the same bits (watertight shared edges).
void cbth::root_triangles(const cbt_mesh* m, std::vector<float>& out)
{
    const int32_t H = m->H;
    out.assign(9 * (size_t)H, 0.0f);
    std::vector<int32_t> face_min(H, -1);
    for (int32_t h = 0; h < H; ++h) {
        if (face_min[h] >= 0) continue;
        int32_t mn = h;
        for (int32_t g = m->next[h]; g != h; g = m->next[g]) mn = g < mn ? g : mn;
        face_min[h] = mn;
        for (int32_t g = m->next[h]; g != h; g = m->next[g]) face_min[g] = mn;
    }
    std::vector<float> centroid(3 * (size_t)H, 0.0f);
    std::vector<uint8_t> done(H, 0);
    for (int32_t h = 0; h < H; ++h) {
        const int32_t f = face_min[h];
        if (done[f]) continue;
        done[f] = 1;
        float sx = m->pos[3 * m->vert[f] + 0], sy = m->pos[3 * m->vert[f] + 1], sz = m->pos[3 * m->vert[f] + 2];
        int n = 1;
        for (int32_t g = m->next[f]; g != f; g = m->next[g]) {
            sx = sx + m->pos[3 * m->vert[g] + 0];
            sy = sy + m->pos[3 * m->vert[g] + 1];
            sz = sz + m->pos[3 * m->vert[g] + 2];
            ++n;
        }
        centroid[3 * f + 0] = sx / (float)n;
        centroid[3 * f + 1] = sy / (float)n;
        centroid[3 * f + 2] = sz / (float)n;
    }
    for (int32_t h = 0; h < H; ++h) {
        const float* a = m->pos + 3 * m->vert[h];
        const float* b = m->pos + 3 * m->vert[m->next[h]];
        const float* c = centroid.data() + 3 * face_min[h];
        for (int i = 0; i < 3; ++i) {
            out[9 * h + i] = a[i];
            out[9 * h + 3 + i] = b[i];
            out[9 * h + 6 + i] = c[i];
        }
    }
}

// The same roots with the face mean accumulated and divided in binary64
// (binary64 instances): corners are the binary32 mesh positions, exact in
// binary64.
static void root_triangles64(const cbt_mesh* m, std::vector<double>& out)
{
    const int32_t H = m->H;
    out.assign(9 * (size_t)H, 0.0);
    for (int32_t h = 0; h < H; ++h) {
        int32_t mn = h;
        for (int32_t g = m->next[h]; g != h; g = m->next[g]) mn = g < mn ? g : mn;
        double sum[3] = {m->pos[3 * m->vert[mn] + 0], m->pos[3 * m->vert[mn] + 1], m->pos[3 * m->vert[mn] + 2]};
        int n = 1;
        for (int32_t g = m->next[mn]; g != mn; g = m->next[g]) {
            for (int i = 0; i < 3; ++i) sum[i] = sum[i] + (double)m->pos[3 * m->vert[g] + i];
            ++n;
        }
        const float* a = m->pos + 3 * m->vert[h];
        const float* b = m->pos + 3 * m->vert[m->next[h]];
        for (int i = 0; i < 3; ++i) {
            out[9 * h + i] = a[i];
            out[9 * h + 3 + i] = b[i];
            out[9 * h + 6 + i] = sum[i] / (double)n;
        }
    }
}

// Device scratch that is free between frames: the work-list region
// (8 bytes per pool block).
static char* list_scratch(const Pool& P, size_t* bytes)
{
    *bytes = sizeof(uint2) * (size_t)P.cap;
    return reinterpret_cast<char*>(P.list);
}

extern "C" {

size_t cbt_workspace_bytes_ex(int32_t H, int32_t D, uint32_t flags)
{
    if (H < 3 || D > 30 || D < ceil_log2(H) || (flags & ~(uint32_t)CBT_INIT_FP64)) return 0;
    return cbtk::workspace_layout(H, D, (flags & CBT_INIT_FP64) ? 1 : 0, nullptr, nullptr);
}

size_t cbt_workspace_bytes(int32_t H, int32_t D) { return cbt_workspace_bytes_ex(H, D, 0); }

cbt_status cbt_init(const cbt_mesh* mesh, int32_t D, void* device_workspace, size_t workspace_bytes,
                    void* hip_stream, cbt_handle* out)
{
    return cbt_init_ex(mesh, D, 0, device_workspace, workspace_bytes, hip_stream, out);
}

// Handle set-up shared by cbt_init_ex and the server's admissions.  With
// base set, the pool receives the base mesh (Section 3.3, "Initialization")
// and the call synchronises; without it (an import of live records follows
// on the same stream, which clears and fills the pool) only the root
// triangles are uploaded, from roots_cached when given (a host array that
// outlives the upload), and nothing waits.
static cbt_status init_impl(const cbt_mesh* mesh, int32_t D, uint32_t flags, void* device_workspace,
                            size_t workspace_bytes, void* hip_stream, cbt_handle* out, bool base,
                            const float* roots_cached, bool validated)
{
    if (!out) return fail(nullptr, CBT_E_ARG, "output handle pointer is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)CBT_INIT_FP64) return fail(nullptr, CBT_E_ARG, "unknown init flags 0x%x", flags);
    const int32_t f64 = (flags & CBT_INIT_FP64) ? 1 : 0;
    if (!validated) {
        cbt_status st = cbth::validate_mesh(mesh);
        if (st) return st;
    }
    const int k = ceil_log2(mesh->H);
    if (D > 30 || D < k) return fail(nullptr, CBT_E_DEPTH, "depth %d outside [ceil(log2 H)=%d, 30]", D, k);
    const size_t need = cbtk::workspace_layout(mesh->H, D, f64, nullptr, nullptr);
    if (!device_workspace) return fail(nullptr, CBT_E_ARG, "device workspace is NULL");
    if (reinterpret_cast<uintptr_t>(device_workspace) & 255) return fail(nullptr, CBT_E_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return fail(nullptr, CBT_E_BUDGET, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    if (roots_cached && f64) return fail(nullptr, CBT_E_ARG, "cached root triangles are binary32");

    cbt_instance* h = new (std::nothrow) cbt_instance();
    if (!h) return fail(nullptr, CBT_E_ARG, "out of host memory");
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, CBT_E_DEVICE, "no current HIP device");
    }
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->ws = reinterpret_cast<char*>(device_workspace);
    h->ws_bytes = workspace_bytes;
    cbtk::workspace_layout(mesh->H, D, f64, &h->P, h->ws);
    h->P.k = k;
    h->P.G = cbth::default_rank_groups(D);
    h->P.sub = cbtk::kMaxReduceSub;
    h->hctr = cbth::pinned_counters();
    if (!h->hctr) {
        delete h;
        return fail(nullptr, CBT_E_DEVICE, "pinned host allocation failed");
    }
    std::memset(h->hctr, 0, sizeof(Counters));
    std::memset(&h->wk, 0, sizeof h->wk);   // flat world positions until LOD parameters arrive

    const int32_t H = mesh->H;
    std::vector<float> roots;
    std::vector<double> roots64;
    if (!roots_cached) {
        if (f64) root_triangles64(mesh, roots64);
        else cbth::root_triangles(mesh, roots);
    }
    const void* root_src = roots_cached ? static_cast<const void*>(roots_cached)
                           : f64        ? static_cast<const void*>(roots64.data())
                                        : static_cast<const void*>(roots.data());
    const size_t root_bytes = 9 * (size_t)H * (f64 ? sizeof(double) : sizeof(float));
    const Pool& P = h->P;
    hipStream_t s = h->stream;
    cbt_status rc = CBT_OK;
    std::vector<uint32_t> recs;
#define INIT_TRY(expr, what)                      \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) {                   \
            rc = hip_fail(nullptr, e_, what);     \
            goto init_fail;                       \
        }                                         \
    } while (0)
    INIT_TRY(hipMemcpyAsync(P.root, root_src, root_bytes, hipMemcpyHostToDevice, s), "upload root triangles");
    if (base) {
        // roots in blocks 0..H-1, packed as (id low, id high, twin, next,
        // prev) and staged in the vertex-cache region (48 bytes per block,
        // cap >= H); the bitfield follows from the IDs
        recs.resize(5 * (size_t)H);
        for (int32_t i = 0; i < H; ++i) {
            const uint64_t id = (uint64_t(1) << k) + (uint64_t)i;
            recs[5 * (size_t)i + 0] = (uint32_t)id;
            recs[5 * (size_t)i + 1] = (uint32_t)(id >> 32);
            recs[5 * (size_t)i + 2] = (uint32_t)mesh->twin[i];
            recs[5 * (size_t)i + 3] = (uint32_t)mesh->next[i];
            recs[5 * (size_t)i + 4] = (uint32_t)mesh->prev[i];
        }
        uint32_t* staging = reinterpret_cast<uint32_t*>(P.vworld);
        INIT_TRY(cbtk::launch_clear_pool(P, s), "clear pool");
        INIT_TRY(hipMemcpyAsync(staging, recs.data(), sizeof(uint32_t) * recs.size(), hipMemcpyHostToDevice, s),
                 "upload roots");
        INIT_TRY(cbtk::launch_import_records(P, 0, (uint32_t)H, staging, s), "root records");
        INIT_TRY(cbtk::launch_bits_from_ids(P, s), "bitfield");
        INIT_TRY(cbtk::launch_reduce(cbtk::single_launch(P, h->wk, nullptr), s), "sum reduction");
        INIT_TRY(cbtk::launch_refresh(cbtk::single_launch(P, h->wk, nullptr), s, true), "vertex cache");
        INIT_TRY(hipStreamSynchronize(s), "init synchronise");
    } else if (!roots_cached) {
        INIT_TRY(hipStreamSynchronize(s), "init synchronise");   // the local root array goes out of scope
    }
#undef INIT_TRY
    *out = h;
    return CBT_OK;
init_fail:
    (void)hipStreamSynchronize(s);
    cbth::release_counters(h->hctr);
    delete h;
    return rc;
}

cbt_status cbt_init_ex(const cbt_mesh* mesh, int32_t D, uint32_t flags, void* device_workspace,
                       size_t workspace_bytes, void* hip_stream, cbt_handle* out)
{
    return init_impl(mesh, D, flags, device_workspace, workspace_bytes, hip_stream, out, true, nullptr, false);
}

static cbt_status read_counters(cbt_handle h)
{
    HIP_TRY(h, hipMemcpyAsync(h->hctr, h->P.ctr, sizeof(Counters), hipMemcpyDeviceToHost, h->stream), "read counters");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    if (h->hctr->err) {
        h->failed = 1;
        return fail(h, CBT_E_DEVICE, "device check failed (flags 0x%x)", h->hctr->err);
    }
    return CBT_OK;
}

// the event pair for this update's timed stage, or NULL
static const cbtk::StageEvents* next_events(cbt_handle h)
{
    thread_local cbtk::StageEvents ev;
    if (!h->timed_stage || h->n_timed >= kMaxTimed) return nullptr;
    const size_t i = 2 * (size_t)h->n_timed;
    if (h->events.size() < i + 2) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return nullptr;
        }
        h->events.push_back(a);
        h->events.push_back(b);
    }
    ev.stage = h->timed_stage;
    ev.begin = h->events[i];
    ev.end = h->events[i + 1];
    h->n_timed++;
    return &ev;
}

static cbt_status finish_frame(cbt_handle h, cbt_frame_stats* stats)
{
    h->last_frame_valid = 1;
    if (!stats) return CBT_OK;
    cbt_status st = read_counters(h);
    if (st) return st;
    return cbth::stats_from_counters(h, *h->hctr, stats);
}

cbt_status cbt_update(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod, cbt_frame_stats* stats)
{
    if (!h) return fail(nullptr, CBT_E_ARG, "NULL handle");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    cbt_status st = cbth::check_lod(h, camera, lod);
    if (st) return st;
    LodK K;
    cbth::make_lodk(camera, lod, &K);
    if (cbth::world_changed(K, h->wk)) {
        // new world-position parameters: recompute the cached world positions
        h->wk = K;
        HIP_TRY(h, cbtk::launch_refresh(cbtk::single_launch(h->P, K, nullptr), h->stream, false), "vertex cache");
    }
    HIP_TRY(h, cbtk::launch_frame(cbtk::single_launch(h->P, K, nullptr), h->stream, next_events(h)), "frame launch");
    return finish_frame(h, stats);
}

// ---------------------------------------------------------------------------
// cbt_update_noalloc: the frame with its scratch arrays (rank list, free
// list, work lists, owner offsets, list lengths, partial sums, statistics
// lanes) in static device memory instead of the handle's workspace, so the
// call allocates nothing.  One copy per GPU, kept until the process ends.
// ---------------------------------------------------------------------------

static constexpr int32_t kNoallocMaxD = 20;
static constexpr size_t kNoallocBlocks = size_t(1) << kNoallocMaxD;
static constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
static constexpr size_t kNoallocLive = 0;
static constexpr size_t kNoallocFree = kNoallocLive + al256(4 * kNoallocBlocks);
static constexpr size_t kNoallocList = kNoallocFree + al256(4 * kNoallocBlocks);
static constexpr size_t kNoallocLpre = kNoallocList + al256(8 * kNoallocBlocks);
static constexpr size_t kNoallocLcnt = kNoallocLpre + al256(4 * kNoallocBlocks);
static constexpr size_t kNoallocPart = kNoallocLcnt + al256(4 * (size_t)cbtk::kMaxRankGroups);
static constexpr size_t kNoallocLane = kNoallocPart + al256(sizeof(uint2) * cbtk::kMaxRankGroups);
static constexpr size_t kNoallocBytes = kNoallocLane + al256(4 * (size_t)cbtk::kStLanes * cbtk::kLaneWords);

// In host code this name is a stand-in, not a device address: kernels and
// copies get the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

static constexpr int kNoallocDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kNoallocDevices];

// the device address of this GPU's scratch array, looked up once per device
// with that device current
static hipError_t noalloc_scratch(int dev, char** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t cbt_noalloc_scratch_bytes(void) { return kNoallocBytes; }

cbt_status cbt_update_noalloc(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod,
                              cbt_frame_stats* stats)
{
    if (!h) return fail(nullptr, CBT_E_ARG, "NULL handle");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    if (h->P.D > kNoallocMaxD)
        return fail(h, CBT_E_CAPACITY, "cbt_update_noalloc: depth %d exceeds its static scratch (depth <= %d, %zu bytes)",
                    h->P.D, kNoallocMaxD, kNoallocBytes);
    cbt_status st = cbth::check_lod(h, camera, lod);
    if (st) return st;
    int dev = -1;
    HIP_TRY(h, hipGetDevice(&dev), "current device");
    if (dev != h->device)
        return fail(h, CBT_E_ARG, "cbt_update_noalloc: device %d is current, the handle's is %d", dev, h->device);
    if (dev < 0 || dev >= kNoallocDevices)
        return fail(h, CBT_E_ARG, "cbt_update_noalloc: device %d beyond the %d supported", dev, kNoallocDevices);
    char* base = nullptr;
    HIP_TRY(h, noalloc_scratch(dev, &base), "static scratch address");
    Pool Q = h->P;
    Q.live = reinterpret_cast<uint32_t*>(base + kNoallocLive);
    Q.freel = reinterpret_cast<uint32_t*>(base + kNoallocFree);
    Q.list = reinterpret_cast<uint2*>(base + kNoallocList);
    Q.lpre = reinterpret_cast<uint32_t*>(base + kNoallocLpre);
    Q.lcnt = reinterpret_cast<uint32_t*>(base + kNoallocLcnt);
    Q.part = reinterpret_cast<uint2*>(base + kNoallocPart);
    Q.slane = reinterpret_cast<uint32_t*>(base + kNoallocLane);
    LodK K;
    cbth::make_lodk(camera, lod, &K);
    // the statistics lanes must start at zero; the last call on this GPU may
    // have been another instance's, or may have stopped part way
    HIP_TRY(h, cbtk::launch_clear_frame_scratch(Q, h->stream), "clear scratch");
    if (cbth::world_changed(K, h->wk)) {
        h->wk = K;
        HIP_TRY(h, cbtk::launch_refresh(cbtk::single_launch(Q, K, nullptr), h->stream, false), "vertex cache");
    }
    HIP_TRY(h, cbtk::launch_frame(cbtk::single_launch(Q, K, nullptr), h->stream, nullptr), "frame launch");
    // the frame's rank list lives in the shared scratch, not in the handle
    h->last_frame_valid = 0;
    if (!stats) return CBT_OK;
    st = read_counters(h);
    if (st) return st;
    return cbth::stats_from_counters(h, *h->hctr, stats);
}

cbt_status cbt_update_with_decisions(cbt_handle h, const uint8_t* device_decisions, cbt_frame_stats* stats)
{
    if (!h) return fail(nullptr, CBT_E_ARG, "NULL handle");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    if (!device_decisions) return fail(h, CBT_E_ARG, "decision array is NULL");
    // new vertices keep the cached world-position parameters
    HIP_TRY(h, cbtk::launch_frame(cbtk::single_launch(h->P, h->wk, device_decisions), h->stream, next_events(h)),
            "frame launch");
    return finish_frame(h, stats);
}

cbt_status cbt_update_converge(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod, int32_t max_passes,
                               int32_t* passes, cbt_frame_stats* last)
{
    if (!h || !passes) return fail(h, CBT_E_ARG, "NULL argument");
    if (max_passes < 1) return fail(h, CBT_E_ARG, "max_passes %d < 1", max_passes);
    *passes = 0;
    cbt_frame_stats st;
    for (int32_t p = 0; p < max_passes; ++p) {
        cbt_status rc = cbt_update(h, camera, lod, &st);
        if (rc) return rc;
        *passes = p + 1;
        if (st.allocations == 0 && st.frees == 0) break;
    }
    if (last) *last = st;
    return CBT_OK;
}

cbt_status cbt_export_triangles(cbt_handle h, float* device_out, int64_t capacity, int64_t* count)
{
    if (!h || !count || capacity < 0 || (capacity > 0 && !device_out)) return fail(h, CBT_E_ARG, "invalid argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    h->last_frame_valid = 0;
    HIP_TRY(h, cbtk::launch_enumerate(cbtk::single_launch(P, h->wk, nullptr), h->stream), "enumerate");
    cbt_status st = read_counters(h);
    if (st) return st;
    const uint32_t L = h->hctr->L;
    *count = L;
    if (capacity < (int64_t)L) return fail(h, CBT_E_CAPACITY, "capacity %lld < %u live bisectors", (long long)capacity, L);
    const cbtk::StageEvents* ev = h->timed_stage == CBT_STAGE_EXPORT ? next_events(h) : nullptr;
    if (ev) HIP_TRY(h, hipEventRecord(ev->begin, h->stream), "event");
    HIP_TRY(h, cbtk::launch_export_triangles(P, L, device_out, h->stream), "export triangles");
    if (ev) HIP_TRY(h, hipEventRecord(ev->end, h->stream), "event");
    return CBT_OK;
}

cbt_status cbt_set_schedule(cbt_handle h, int32_t rank_groups, int32_t reduce_levels)
{
    if (!h) return fail(nullptr, CBT_E_ARG, "NULL handle");
    if (rank_groups < cbtk::kMinRankGroups || rank_groups > cbtk::kMaxRankGroups)
        return fail(h, CBT_E_ARG, "rank_groups %d outside [%d, %d]", rank_groups, cbtk::kMinRankGroups, cbtk::kMaxRankGroups);
    if (reduce_levels < cbtk::kMinReduceSub || reduce_levels > cbtk::kMaxReduceSub)
        return fail(h, CBT_E_ARG, "reduce_levels %d outside [%d, %d]", reduce_levels, cbtk::kMinReduceSub, cbtk::kMaxReduceSub);
    h->P.G = (uint32_t)rank_groups;
    h->P.sub = reduce_levels;
    return CBT_OK;
}

cbt_status cbt_get_schedule(cbt_handle h, int32_t* rank_groups, int32_t* reduce_levels)
{
    if (!h || !rank_groups || !reduce_levels) return fail(h, CBT_E_ARG, "NULL argument");
    *rank_groups = (int32_t)h->P.G;
    *reduce_levels = h->P.sub;
    return CBT_OK;
}

cbt_status cbt_time_stage(cbt_handle h, int32_t stage)
{
    if (!h) return fail(nullptr, CBT_E_ARG, "NULL handle");
    if (stage < CBT_STAGE_NONE || stage > CBT_STAGE_EXPORT) return fail(h, CBT_E_ARG, "unknown stage %d", stage);
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    h->timed_stage = stage;
    h->n_timed = 0;
    return CBT_OK;
}

cbt_status cbt_stage_time(cbt_handle h, int64_t* launches, double* total_ms)
{
    if (!h || !launches || !total_ms) return fail(h, CBT_E_ARG, "NULL argument");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    double sum = 0.0;
    for (int i = 0; i < h->n_timed; ++i) {
        float ms = 0.0f;
        HIP_TRY(h, hipEventElapsedTime(&ms, h->events[2 * (size_t)i], h->events[2 * (size_t)i + 1]), "event time");
        sum += ms;
    }
    *launches = h->n_timed;
    *total_ms = sum;
    return CBT_OK;
}

cbt_status cbt_stage_times(cbt_handle h, double* out_ms, int64_t capacity, int64_t* count)
{
    if (!h || !count || (capacity > 0 && !out_ms) || capacity < 0) return fail(h, CBT_E_ARG, "invalid argument");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    *count = h->n_timed;
    if (capacity < h->n_timed) return fail(h, CBT_E_CAPACITY, "capacity %lld < %d timed launches", (long long)capacity, h->n_timed);
    for (int i = 0; i < h->n_timed; ++i) {
        float ms = 0.0f;
        HIP_TRY(h, hipEventElapsedTime(&ms, h->events[2 * (size_t)i], h->events[2 * (size_t)i + 1]), "event time");
        out_ms[i] = ms;
    }
    return CBT_OK;
}

cbt_status cbt_live_count(cbt_handle h, int64_t* out)
{
    if (!h || !out) return fail(h, CBT_E_ARG, "NULL argument");
    uint32_t L = 0;
    HIP_TRY(h, hipMemcpyAsync(&L, h->P.tree + 1, sizeof L, hipMemcpyDeviceToHost, h->stream), "read root");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    *out = L;
    return CBT_OK;
}

cbt_status cbt_query(cbt_handle h, cbt_bisectors* out)
{
    if (!h || !out) return fail(h, CBT_E_ARG, "NULL argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    hipStream_t s = h->stream;
    h->last_frame_valid = 0;
    HIP_TRY(h, cbtk::launch_enumerate(cbtk::single_launch(P, h->wk, nullptr), s), "enumerate");
    cbt_status st = read_counters(h);
    if (st) return st;
    const uint32_t L = h->hctr->L;
    out->count = L;
    const bool per = out->slot || out->heap_id || out->twin || out->next || out->prev || out->vertices || out->vertices64 ||
                     out->root_h || out->subdiv_id;
    if (per && out->capacity < (int64_t)L) return fail(h, CBT_E_CAPACITY, "capacity %lld < %u live bisectors", (long long)out->capacity, L);
    size_t scratch_bytes;
    char* scratch = list_scratch(P, &scratch_bytes);
    if (out->slot && L)
        HIP_TRY(h, hipMemcpyAsync(out->slot, P.live, sizeof(uint32_t) * L, hipMemcpyDeviceToHost, s), "copy slots");
    if (out->heap_id && L) {
        HIP_TRY(h, cbtk::launch_gather_ids(P, 0, L, reinterpret_cast<uint64_t*>(scratch), s), "gather IDs");
        HIP_TRY(h, hipMemcpyAsync(out->heap_id, scratch, sizeof(uint64_t) * L, hipMemcpyDeviceToHost, s), "copy IDs");
        HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
    }
    if (out->root_h && L) {
        HIP_TRY(h, cbtk::launch_gather_canonical(P, 0, L, reinterpret_cast<int32_t*>(scratch), nullptr, s), "gather roots");
        HIP_TRY(h, hipMemcpyAsync(out->root_h, scratch, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s), "copy roots");
        HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
    }
    if (out->subdiv_id && L) {
        HIP_TRY(h, cbtk::launch_gather_canonical(P, 0, L, nullptr, reinterpret_cast<uint64_t*>(scratch), s), "gather codes");
        HIP_TRY(h, hipMemcpyAsync(out->subdiv_id, scratch, sizeof(uint64_t) * L, hipMemcpyDeviceToHost, s), "copy codes");
        HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
    }
    if ((out->twin || out->next || out->prev) && L) {
        std::vector<int32_t> tmp(3 * (size_t)L);
        const uint32_t chunk = (uint32_t)(scratch_bytes / (3 * sizeof(int32_t)));
        for (uint32_t r0 = 0; r0 < L; r0 += chunk) {
            const uint32_t n = (L - r0) < chunk ? (L - r0) : chunk;
            HIP_TRY(h, cbtk::launch_gather_links(P, r0, n, reinterpret_cast<int32_t*>(scratch), s), "gather links");
            HIP_TRY(h, hipMemcpyAsync(tmp.data() + 3 * (size_t)r0, scratch, sizeof(int32_t) * 3 * n, hipMemcpyDeviceToHost, s),
                    "copy links");
            HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
        }
        for (uint32_t i = 0; i < L; ++i) {
            if (out->twin) out->twin[i] = tmp[3 * (size_t)i];
            if (out->next) out->next[i] = tmp[3 * (size_t)i + 1];
            if (out->prev) out->prev[i] = tmp[3 * (size_t)i + 2];
        }
    }
    if (out->vertices && L) {
        const uint32_t chunk = (uint32_t)(scratch_bytes / (9 * sizeof(float)));
        for (uint32_t r0 = 0; r0 < L; r0 += chunk) {
            const uint32_t n = (L - r0) < chunk ? (L - r0) : chunk;
            HIP_TRY(h, cbtk::launch_gather_vertices(P, r0, n, reinterpret_cast<float*>(scratch), s), "gather vertices");
            HIP_TRY(h, hipMemcpyAsync(out->vertices + 9 * (size_t)r0, scratch, sizeof(float) * 9 * n, hipMemcpyDeviceToHost, s),
                    "copy vertices");
            HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
        }
    }
    if (out->vertices64 && L) {
        const uint32_t chunk = (uint32_t)(scratch_bytes / (9 * sizeof(double)));
        for (uint32_t r0 = 0; r0 < L; r0 += chunk) {
            const uint32_t n = (L - r0) < chunk ? (L - r0) : chunk;
            HIP_TRY(h, cbtk::launch_gather_vertices64(P, r0, n, reinterpret_cast<double*>(scratch), s), "gather vertices");
            HIP_TRY(h, hipMemcpyAsync(out->vertices64 + 9 * (size_t)r0, scratch, sizeof(double) * 9 * n, hipMemcpyDeviceToHost, s),
                    "copy vertices");
            HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
        }
    }
    if (out->tree) {
        static_assert(sizeof(uint2) == 2 * sizeof(uint32_t), "scratch holds the 2^(D+1) heap");
        HIP_TRY(h, cbtk::launch_export_heap(P, reinterpret_cast<uint32_t*>(scratch), s), "export tree");
        HIP_TRY(h, hipMemcpyAsync(out->tree, scratch, sizeof(uint32_t) * 2 * (size_t)P.cap, hipMemcpyDeviceToHost, s), "copy tree");
    }
    HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
    return CBT_OK;
}

cbt_status cbt_query_decisions(cbt_handle h, uint8_t* per_slot)
{
    if (!h || !per_slot) return fail(h, CBT_E_ARG, "NULL argument");
    if (!h->last_frame_valid) return fail(h, CBT_E_STATE, "no frame since the last query");
    const Pool& P = h->P;
    cbt_status st = read_counters(h);
    if (st) return st;
    uint8_t* dec = reinterpret_cast<uint8_t*>(P.freel);   // 4 * cap bytes, free between frames
    HIP_TRY(h, cbtk::launch_gather_decisions(P, h->hctr->L, dec, h->stream), "gather decisions");
    HIP_TRY(h, hipMemcpyAsync(per_slot, dec, P.cap, hipMemcpyDeviceToHost, h->stream), "copy decisions");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    return CBT_OK;
}

cbt_status cbt_snapshot(cbt_handle h, uint64_t* heap_id, int32_t* twin, int32_t* next, int32_t* prev)
{
    if (!h || !heap_id || !twin || !next || !prev) return fail(h, CBT_E_ARG, "NULL argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    size_t scratch_bytes;
    uint32_t* scratch = reinterpret_cast<uint32_t*>(list_scratch(P, &scratch_bytes));
    const uint32_t chunk = (uint32_t)(scratch_bytes / (5 * sizeof(uint32_t)));
    std::vector<uint32_t> recs(5 * (size_t)P.cap);
    std::vector<uint32_t> words(P.W);
    HIP_TRY(h, hipMemcpyAsync(words.data(), P.bits, sizeof(uint32_t) * P.W, hipMemcpyDeviceToHost, h->stream), "copy bits");
    for (uint32_t b0 = 0; b0 < P.cap; b0 += chunk) {
        const uint32_t n = (P.cap - b0) < chunk ? (P.cap - b0) : chunk;
        HIP_TRY(h, cbtk::launch_export_records(P, b0, n, scratch, h->stream), "export records");
        HIP_TRY(h, hipMemcpyAsync(recs.data() + 5 * (size_t)b0, scratch, sizeof(uint32_t) * 5 * n, hipMemcpyDeviceToHost,
                                  h->stream), "copy records");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    }
    for (uint32_t i = 0; i < P.cap; ++i) {
        const bool live = (words[i >> 5] >> (i & 31)) & 1u;
        const uint32_t* r = recs.data() + 5 * (size_t)i;
        heap_id[i] = live ? ((uint64_t)r[0] | ((uint64_t)r[1] << 32)) : 0;
        twin[i] = live ? (int32_t)r[2] : -1;
        next[i] = live ? (int32_t)r[3] : -1;
        prev[i] = live ? (int32_t)r[4] : -1;
    }
    h->last_frame_valid = 0;
    return CBT_OK;
}

cbt_status cbt_restore(cbt_handle h, const uint64_t* heap_id, const int32_t* twin, const int32_t* next,
                       const int32_t* prev)
{
    if (!h || !heap_id || !twin || !next || !prev) return fail(h, CBT_E_ARG, "NULL argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    std::vector<uint32_t> recs(5 * (size_t)P.cap);
    for (uint32_t i = 0; i < P.cap; ++i) {
        uint32_t* r = recs.data() + 5 * (size_t)i;
        r[0] = (uint32_t)heap_id[i];
        r[1] = (uint32_t)(heap_id[i] >> 32);
        if (heap_id[i]) {
            const int32_t t = twin[i], n = next[i], p = prev[i];
            if (t < -1 || t >= (int64_t)P.cap || n < -1 || n >= (int64_t)P.cap || p < -1 || p >= (int64_t)P.cap)
                return fail(h, CBT_E_ARG, "restore: pointer of slot %u out of range", i);
            r[2] = (uint32_t)t;
            r[3] = (uint32_t)n;
            r[4] = (uint32_t)p;
        } else {
            r[2] = r[3] = r[4] = 0xffffffffu;
        }
    }
    size_t scratch_bytes;
    uint32_t* scratch = reinterpret_cast<uint32_t*>(list_scratch(P, &scratch_bytes));
    const uint32_t chunk = (uint32_t)(scratch_bytes / (5 * sizeof(uint32_t)));
    for (uint32_t b0 = 0; b0 < P.cap; b0 += chunk) {
        const uint32_t n = (P.cap - b0) < chunk ? (P.cap - b0) : chunk;
        HIP_TRY(h, hipMemcpyAsync(scratch, recs.data() + 5 * (size_t)b0, sizeof(uint32_t) * 5 * n, hipMemcpyHostToDevice,
                                  h->stream), "upload records");
        HIP_TRY(h, cbtk::launch_import_records(P, b0, n, scratch, h->stream), "import records");
        HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    }
    const cbtk::Launch X = cbtk::single_launch(P, h->wk, nullptr);
    HIP_TRY(h, cbtk::launch_bits_from_ids(P, h->stream), "bitfield");
    HIP_TRY(h, cbtk::launch_reduce(X, h->stream), "sum reduction");
    HIP_TRY(h, cbtk::launch_refresh(X, h->stream, true), "vertex cache");
    HIP_TRY(h, hipStreamSynchronize(h->stream), "synchronise");
    h->last_frame_valid = 0;
    return CBT_OK;
}

cbt_status cbt_export_live(cbt_handle h, uint32_t* records, int64_t capacity, int64_t* count)
{
    if (!h || !count) return fail(h, CBT_E_ARG, "NULL argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    HIP_TRY(h, cbtk::launch_enumerate(cbtk::single_launch(P, h->wk, nullptr), h->stream), "enumerate");
    cbt_status st = read_counters(h);
    if (st) return st;
    const uint32_t L = h->hctr->L;
    *count = L;
    if (capacity < (int64_t)L) return fail(h, CBT_E_CAPACITY, "capacity %lld < %u live bisectors", (long long)capacity, L);
    if (!records) return fail(h, CBT_E_ARG, "NULL records");
    HIP_TRY(h, cbtk::launch_export_live(P, L, records, h->stream, false), "export live records");
    return CBT_OK;
}

cbt_status cbt_import_live(cbt_handle h, const uint32_t* records, int64_t count, int32_t on_host)
{
    if (!h || !records) return fail(h, CBT_E_ARG, "NULL argument");
    if (h->failed) return fail(h, CBT_E_STATE, "handle failed earlier: %s", h->err);
    const Pool& P = h->P;
    if (count < 1 || count > (int64_t)P.cap) return fail(h, CBT_E_ARG, "record count %lld outside [1, 2^D]", (long long)count);
    hipStream_t s = h->stream;
    HIP_TRY(h, cbtk::launch_clear_pool(P, s), "clear pool");
    if (on_host) {
        size_t scratch_bytes;
        uint32_t* scratch = reinterpret_cast<uint32_t*>(list_scratch(P, &scratch_bytes));
        const uint32_t chunk = (uint32_t)(scratch_bytes / (6 * sizeof(uint32_t)));
        for (int64_t r0 = 0; r0 < count; r0 += chunk) {
            const uint32_t n = (uint32_t)((count - r0) < chunk ? (count - r0) : chunk);
            HIP_TRY(h, hipMemcpyAsync(scratch, records + 6 * r0, sizeof(uint32_t) * 6 * n, hipMemcpyHostToDevice, s),
                    "upload records");
            HIP_TRY(h, cbtk::launch_import_live(P, n, scratch, s), "import live records");
            HIP_TRY(h, hipStreamSynchronize(s), "synchronise");
        }
    } else {
        HIP_TRY(h, cbtk::launch_import_live(P, (uint32_t)count, records, s), "import live records");
    }
    const cbtk::Launch X = cbtk::single_launch(P, h->wk, nullptr);
    HIP_TRY(h, cbtk::launch_bits_from_ids(P, s), "bitfield");
    HIP_TRY(h, cbtk::launch_reduce(X, s), "sum reduction");
    HIP_TRY(h, cbtk::launch_refresh(X, s, true), "vertex cache");
    h->last_frame_valid = 0;
    return read_counters(h);
}

cbt_status cbt_frame_constants(cbt_handle h, const cbt_camera* camera, const cbt_lod_params* lod, float* out18)
{
    if (!out18) return fail(h, CBT_E_ARG, "NULL output");
    cbt_lod_params lp = lod ? *lod : cbt_lod_params{CBT_MODE_FLAT, 1.0f, 1.0f, nullptr, 0, 0.0f, CBT_CRIT_EDGE};
    lp.mode = CBT_MODE_FLAT;   // the table is irrelevant for the constants
    cbt_status st = cbth::check_lod(h, camera, &lp);
    if (st) return st;
    LodK K;
    cbth::make_lodk(camera, &lp, &K);
    const double v[18] = {K.cam[0], K.cam[1], K.cam[2], K.right[0], K.right[1], K.right[2], K.up[0], K.up[1], K.up[2],
                          K.fwd[0], K.fwd[1], K.fwd[2], K.f2, K.t2s, K.t2m, K.tx, K.ty, K.znear};
    for (int i = 0; i < 18; ++i) out18[i] = (float)v[i];   // the binary32 path's constants
    return CBT_OK;
}

cbt_status cbt_destroy(cbt_handle h)
{
    if (!h) return CBT_OK;
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    cbth::release_counters(h->hctr);
    delete h;
    return CBT_OK;
}

const char* cbt_status_string(cbt_status s)
{
    switch (s) {
    case CBT_OK: return "ok";
    case CBT_E_ARG: return "invalid argument";
    case CBT_E_MESH: return "invalid mesh";
    case CBT_E_DEPTH: return "invalid depth";
    case CBT_E_CAPACITY: return "output capacity too small";
    case CBT_E_DEVICE: return "device error";
    case CBT_E_BUDGET: return "workspace too small";
    case CBT_E_STATE: return "handle in a failed state";
    default: return "unknown status";
    }
}

const char* cbt_last_error(cbt_handle h) { return h ? h->err : g_err; }

}  // extern "C"

cbt_status cbth::init_for_import(const cbt_mesh* mesh, int32_t D, void* device_workspace, size_t workspace_bytes,
                                 void* hip_stream, const float* roots, cbt_handle* out)
{
    return init_impl(mesh, D, 0, device_workspace, workspace_bytes, hip_stream, out, false, roots, true);
}
