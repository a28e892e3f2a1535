// Batched update: many instances (uneven meshes and depths) advanced by one
// launch per pipeline stage.  Each instance keeps its own workspace and
// counters; the batch adds, in a workspace of its own, the instance
// descriptors and three block maps that send every workgroup of a batched
// grid to its instance.  The launch sequence can be captured once as a HIP
// graph and replayed every frame: the per-frame constants reach the device
// through the descriptor upload that precedes each replay.

#include "cbt_host.h"

#include <cstring>
#include <new>
#include <vector>

using cbtk::Counters;
using cbtk::Inst;
using cbtk::LodK;
using cbtk::Pool;

struct cbt_batch_s {
    std::vector<cbt_handle> m;
    std::vector<Pool> pools;    // member state and schedule as of creation
    int n;
    hipStream_t stream;
    Inst* d_inst;
    Counters* d_ctr;
    uint32_t *d_map_rank, *d_map_word, *d_map_red, *d_map_list;
    Inst* h_stage[2];           // pinned descriptor staging, double-buffered
    hipEvent_t staged[2];       // the upload from that buffer has completed
    bool stage_used[2];
    int cur;
    Counters* h_ctr;            // pinned
    cbtk::Launch X;
    bool use_graph;
    bool captured;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int failed;
};

namespace {

struct Layout {
    size_t inst, ctr, map_rank, map_word, map_red, map_list, ticket, done, pmap, total;
};

// workgroups of the batched grids: rank, bitfield-word, reduction and
// list; items of the persistent frame
struct Grids {
    uint64_t nr, nw, nd, nl, items;
};

Layout batch_layout(int n, const Grids& g)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    L.inst = take(sizeof(Inst) * (size_t)n);
    L.ctr = take(sizeof(Counters) * (size_t)n);
    L.map_rank = take(4 * g.nr);
    L.map_word = take(4 * g.nw);
    L.map_red = take(4 * g.nd);
    L.map_list = take(4 * g.nl);
    L.ticket = take(4);
    L.done = take(4 * (size_t)n * cbtk::kPhCount);
    L.pmap = take(4 * g.items);
    L.total = off;
    return L;
}

cbt_status check_members(const cbt_handle* members, int32_t n)
{
    if (!members || n < 1 || n > cbtk::kMaxBatch)
        return cbth::fail(nullptr, CBT_E_ARG, "batch needs 1..%d member handles", cbtk::kMaxBatch);
    for (int i = 0; i < n; ++i) {
        if (!members[i]) return cbth::fail(nullptr, CBT_E_ARG, "member %d is NULL", i);
        if (members[i]->failed) return cbth::fail(nullptr, CBT_E_STATE, "member %d failed earlier: %s", i, members[i]->err);
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return cbth::fail(nullptr, CBT_E_ARG, "member %d appears twice", i);
        if (members[i]->P.f64 != members[0]->P.f64)
            return cbth::fail(nullptr, CBT_E_ARG, "member %d: a batch holds instances of one precision", i);
    }
    return CBT_OK;
}

Grids grid_totals(const cbt_handle* members, int32_t n)
{
    Grids g{0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const Pool& P = members[i]->P;
        g.nr += P.G;
        g.nw += cbtk::word_groups(P);
        g.nd += cbtk::reduce_groups(P);
        g.nl += cbtk::list_groups(P);
        for (int p = 0; p < cbtk::kPhCount; ++p) g.items += cbtk::persist_items_host(cbtk::phase_groups_host(P, p));
    }
    return g;
}

cbt_status batch_fail(cbt_batch b, hipError_t e, const char* what)
{
    if (b) b->failed = 1;
    return cbth::fail(nullptr, CBT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define BATCH_TRY(b, expr, what)                             \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return batch_fail(b, e_, what); \
    } while (0)

// Descriptors for this frame: upload through the staging buffer not used by
// the previous frame (its last upload has completed before it is rewritten).
cbt_status upload_descriptors(cbt_batch b, const std::vector<LodK>& K, const uint8_t* const* inj)
{
    const int c = b->cur;
    if (b->stage_used[c]) BATCH_TRY(b, hipEventSynchronize(b->staged[c]), "staging wait");
    Inst* st = b->h_stage[c];
    for (int i = 0; i < b->n; ++i) {
        st[i].P = b->pools[i];
        st[i].K = K[i];
        st[i].inj = inj ? inj[i] : nullptr;
    }
    BATCH_TRY(b, hipMemcpyAsync(b->d_inst, st, sizeof(Inst) * (size_t)b->n, hipMemcpyHostToDevice, b->stream),
              "descriptor upload");
    BATCH_TRY(b, hipEventRecord(b->staged[c], b->stream), "staging event");
    b->stage_used[c] = true;
    b->cur ^= 1;
    return CBT_OK;
}

cbt_status run_frame(cbt_batch b)
{
    if (!b->use_graph) {
        BATCH_TRY(b, cbtk::launch_frame(b->X, b->stream, nullptr), "batched frame");
        return CBT_OK;
    }
    if (!b->captured) {
        BATCH_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t e = cbtk::launch_frame(b->X, b->stream, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return batch_fail(b, e, "capture launches");
        }
        BATCH_TRY(b, e2, "end capture");
        b->graph = g;
        BATCH_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        b->captured = true;
    }
    BATCH_TRY(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
    return CBT_OK;
}

cbt_status finish(cbt_batch b, cbt_frame_stats* stats)
{
    for (int i = 0; i < b->n; ++i) b->m[i]->last_frame_valid = 1;
    if (!stats) return CBT_OK;
    BATCH_TRY(b, cbtk::launch_gather_counters(b->X, b->d_ctr, b->stream), "gather counters");
    BATCH_TRY(b, hipMemcpyAsync(b->h_ctr, b->d_ctr, sizeof(Counters) * (size_t)b->n, hipMemcpyDeviceToHost, b->stream),
              "copy counters");
    BATCH_TRY(b, hipStreamSynchronize(b->stream), "synchronise");
    cbt_status rc = CBT_OK;
    for (int i = 0; i < b->n; ++i) {
        cbt_status st = cbth::stats_from_counters(b->m[i], b->h_ctr[i], &stats[i]);
        if (st && rc == CBT_OK) {
            rc = cbth::fail(nullptr, st, "member %d: %s", i, b->m[i]->err);
            b->failed = 1;
        }
    }
    return rc;
}

}  // namespace

extern "C" {

size_t cbt_batch_workspace_bytes(const cbt_handle* members, int32_t n)
{
    if (check_members(members, n) != CBT_OK) return 0;
    return batch_layout(n, grid_totals(members, n)).total;
}

cbt_status cbt_batch_create(const cbt_handle* members, int32_t n, void* device_workspace, size_t workspace_bytes,
                            void* hip_stream, int32_t flags, cbt_batch* out)
{
    if (!out) return cbth::fail(nullptr, CBT_E_ARG, "output batch pointer is NULL");
    *out = nullptr;
    cbt_status st = check_members(members, n);
    if (st) return st;
    if (flags & ~(CBT_BATCH_GRAPH | CBT_BATCH_PERSISTENT))
        return cbth::fail(nullptr, CBT_E_ARG, "unknown batch flags 0x%x", flags);
    if ((flags & CBT_BATCH_GRAPH) && !hip_stream)
        return cbth::fail(nullptr, CBT_E_ARG, "graph capture needs a stream other than the null stream");
    const Grids gt = grid_totals(members, n);
    const Layout L = batch_layout(n, gt);
    if (!device_workspace) return cbth::fail(nullptr, CBT_E_ARG, "device workspace is NULL");
    if (reinterpret_cast<uintptr_t>(device_workspace) & 255)
        return cbth::fail(nullptr, CBT_E_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return cbth::fail(nullptr, CBT_E_BUDGET, "batch workspace has %zu bytes, needs %zu", workspace_bytes, L.total);

    cbt_batch b = new (std::nothrow) cbt_batch_s();
    if (!b) return cbth::fail(nullptr, CBT_E_ARG, "out of host memory");
    b->n = n;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->use_graph = (flags & CBT_BATCH_GRAPH) != 0;
    char* ws = reinterpret_cast<char*>(device_workspace);
    b->d_inst = reinterpret_cast<Inst*>(ws + L.inst);
    b->d_ctr = reinterpret_cast<Counters*>(ws + L.ctr);
    b->d_map_rank = reinterpret_cast<uint32_t*>(ws + L.map_rank);
    b->d_map_word = reinterpret_cast<uint32_t*>(ws + L.map_word);
    b->d_map_red = reinterpret_cast<uint32_t*>(ws + L.map_red);
    b->d_map_list = reinterpret_cast<uint32_t*>(ws + L.map_list);
    b->m.assign(members, members + n);
    std::vector<uint32_t> mr, mw, md, ml;
    mr.reserve(gt.nr);
    mw.reserve(gt.nw);
    md.reserve(gt.nd);
    ml.reserve(gt.nl);
    for (int i = 0; i < n; ++i) {
        const Pool& P = members[i]->P;
        b->pools.push_back(P);
        const uint32_t tag = (uint32_t)i << cbtk::kMapShift;
        for (uint32_t g = 0; g < P.G; ++g) mr.push_back(tag | g);
        for (uint32_t g = 0; g < cbtk::word_groups(P); ++g) mw.push_back(tag | g);
        for (uint32_t g = 0; g < cbtk::reduce_groups(P); ++g) md.push_back(tag | g);
        for (uint32_t g = 0; g < cbtk::list_groups(P); ++g) ml.push_back(tag | g);
    }
    cbt_status rc = CBT_OK;
    auto bail = [&](cbt_status s) {
        rc = s;
        return s;
    };
    do {
        bool ok = true;
        for (int c = 0; c < 2 && ok; ++c) {
            ok = hipHostMalloc(reinterpret_cast<void**>(&b->h_stage[c]), sizeof(Inst) * (size_t)n, hipHostMallocDefault) ==
                     hipSuccess &&
                 hipEventCreateWithFlags(&b->staged[c], hipEventDisableTiming) == hipSuccess;
        }
        ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_ctr), sizeof(Counters) * (size_t)n, hipHostMallocDefault) ==
                       hipSuccess;
        if (!ok) {
            bail(cbth::fail(nullptr, CBT_E_DEVICE, "pinned host allocation failed"));
            break;
        }
        // members' earlier work is ordered before the batch's by completing it
        for (int i = 0; i < n && rc == CBT_OK; ++i)
            if (hipStreamSynchronize(members[i]->stream) != hipSuccess)
                bail(cbth::fail(nullptr, CBT_E_DEVICE, "member %d: synchronise", i));
        if (rc) break;
        hipStream_t s = b->stream;
        if (hipMemcpyAsync(b->d_map_rank, mr.data(), 4 * mr.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_map_word, mw.data(), 4 * mw.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_map_red, md.data(), 4 * md.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(b->d_map_list, ml.data(), 4 * ml.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            bail(cbth::fail(nullptr, CBT_E_DEVICE, "block map upload failed"));
            break;
        }
    } while (false);
    if (rc) {
        for (int c = 0; c < 2; ++c) {
            if (b->h_stage[c]) (void)hipHostFree(b->h_stage[c]);
            if (b->staged[c]) (void)hipEventDestroy(b->staged[c]);
        }
        if (b->h_ctr) (void)hipHostFree(b->h_ctr);
        delete b;
        return rc;
    }
    cbtk::Launch& X = b->X;
    std::memset(&X, 0, sizeof X);
    X.batched = true;
    X.f64 = members[0]->P.f64 != 0;
    X.B.n = n;
    X.B.inst = b->d_inst;
    X.B.map_rank = b->d_map_rank;
    X.B.map_word = b->d_map_word;
    X.B.map_red = b->d_map_red;
    X.B.map_list = b->d_map_list;
    X.n_inst = (uint32_t)n;
    X.grid_rank = (uint32_t)gt.nr;
    X.grid_word = (uint32_t)gt.nw;
    X.grid_red = (uint32_t)gt.nd;
    X.grid_list = (uint32_t)gt.nl;
    if (flags & CBT_BATCH_PERSISTENT) {
        // items phase by phase, in each phase instance by instance; an item
        // is a span of the instance's workgroups for the phase
        std::vector<uint32_t> pm;
        pm.reserve(gt.items);
        uint64_t at = 0;
        for (int p = 0; p < cbtk::kPhCount; ++p) {
            X.W.first[p] = (uint32_t)at;
            for (int i = 0; i < n; ++i) {
                const uint32_t k = cbtk::persist_items_host(cbtk::phase_groups_host(b->pools[i], p));
                for (uint32_t t = 0; t < k; ++t) pm.push_back(((uint32_t)i << cbtk::kMapShift) | t);
                at += k;
            }
        }
        X.W.first[cbtk::kPhCount] = (uint32_t)at;
        uint32_t* d_pmap = reinterpret_cast<uint32_t*>(ws + L.pmap);
        if (hipMemcpyAsync(d_pmap, pm.data(), 4 * pm.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess) {
            cbt_status st2 = cbth::fail(nullptr, CBT_E_DEVICE, "persistent work list upload failed");
            cbt_batch_destroy(b);
            return st2;
        }
        X.W.map = d_pmap;
        X.W.fail_phase = cbtk::kPhCount;
        X.W.ticket = reinterpret_cast<uint32_t*>(ws + L.ticket);
        X.W.done = reinterpret_cast<uint32_t*>(ws + L.done);
        const uint32_t resident = cbtk::persist_resident_groups(X.f64);
        X.persistent = true;
        X.persist_groups = resident == 0 ? 256u : (resident < at ? resident : (uint32_t)at);
    }
    *out = b;
    return CBT_OK;
}

cbt_status cbt_batch_update(cbt_batch b, const cbt_camera* cameras, const cbt_lod_params* lods, cbt_frame_stats* stats)
{
    if (!b || !cameras || !lods) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    if (b->failed) return cbth::fail(nullptr, CBT_E_STATE, "batch failed earlier");
    std::vector<LodK> K(b->n);
    for (int i = 0; i < b->n; ++i) {
        cbt_handle h = b->m[i];
        if (h->failed) return cbth::fail(nullptr, CBT_E_STATE, "member %d failed earlier: %s", i, h->err);
        cbt_status st = cbth::check_lod(h, &cameras[i], &lods[i]);
        if (st) return cbth::fail(nullptr, st, "member %d: %s", i, h->err);
        cbth::make_lodk(&cameras[i], &lods[i], &K[i]);
    }
    for (int i = 0; i < b->n; ++i) {
        cbt_handle h = b->m[i];
        if (cbth::world_changed(K[i], h->wk)) {
            h->wk = K[i];
            BATCH_TRY(b, cbtk::launch_refresh(cbtk::single_launch(b->pools[i], K[i], nullptr), b->stream, false),
                      "vertex cache");
        }
    }
    cbt_status st = upload_descriptors(b, K, nullptr);
    if (st) return st;
    st = run_frame(b);
    if (st) return st;
    return finish(b, stats);
}

cbt_status cbt_batch_update_with_decisions(cbt_batch b, const uint8_t* const* device_decisions, cbt_frame_stats* stats)
{
    if (!b || !device_decisions) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    if (b->failed) return cbth::fail(nullptr, CBT_E_STATE, "batch failed earlier");
    std::vector<LodK> K(b->n);
    for (int i = 0; i < b->n; ++i) {
        if (!device_decisions[i]) return cbth::fail(nullptr, CBT_E_ARG, "decision array of member %d is NULL", i);
        if (b->m[i]->failed) return cbth::fail(nullptr, CBT_E_STATE, "member %d failed earlier", i);
        K[i] = b->m[i]->wk;
    }
    cbt_status st = upload_descriptors(b, K, device_decisions);
    if (st) return st;
    st = run_frame(b);
    if (st) return st;
    return finish(b, stats);
}

cbt_status cbt_batch_fail_stage(cbt_batch b, int32_t stage)
{
    if (!b) return cbth::fail(nullptr, CBT_E_ARG, "NULL batch");
    if (!b->X.persistent) return cbth::fail(nullptr, CBT_E_ARG, "not a persistent batch");
    if (stage != -1 && (stage < 1 || stage >= cbtk::kPhCount))
        return cbth::fail(nullptr, CBT_E_ARG, "stage %d outside [1, %d)", stage, (int)cbtk::kPhCount);
    BATCH_TRY(b, hipStreamSynchronize(b->stream), "synchronise");
    b->X.W.fail_phase = stage < 0 ? (uint32_t)cbtk::kPhCount : (uint32_t)stage;
    // the launch arguments live in the captured graph: capture again
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = false;
    return CBT_OK;
}

cbt_status cbt_batch_destroy(cbt_batch b)
{
    if (!b) return CBT_OK;
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int c = 0; c < 2; ++c) {
        if (b->h_stage[c]) (void)hipHostFree(b->h_stage[c]);
        if (b->staged[c]) (void)hipEventDestroy(b->staged[c]);
    }
    if (b->h_ctr) (void)hipHostFree(b->h_ctr);
    delete b;
    return CBT_OK;
}

}  // extern "C"
