// Serving loop: tessellation-update requests (instance, camera) arrive at
// any time; each instance keeps its state resident in device memory while it
// fits, instances are admitted by their workspace footprint against a
// memory budget and idle ones are evicted to host snapshots; requests are
// batched continuously: whenever a launch slot is free, every instance with
// a queued request and none in flight joins the next batched frame, which
// runs on the slot's own stream, so batches of different instances overlap
// on the device.  At most one request per instance is in flight, so each
// instance sees its requests in arrival order and its result is the one it
// gets alone.

#include "cbt_host.h"

#include <cmath>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <new>
#include <unordered_map>
#include <vector>

using cbtk::Counters;
using cbtk::Inst;
using cbtk::LodK;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t tag;
    cbt_camera cam;
    double t_arrive;
};

struct SInst {
    int64_t id = 0;
    std::vector<int32_t> twin, next, prev, vert;
    std::vector<float> pos;
    std::vector<float> roots;   // root triangles, computed once at open
    int32_t H = 0, V = 0, D = 0;
    cbt_lod_params lod{};
    int32_t groups = 0, levels = 0;   // schedule (0: library default)
    cbt_handle h = nullptr;
    size_t off = 0, bytes = 0;
    // state of an evicted instance: its live records (cbt_export_live), in
    // the arena's top end or, when even that is full, on the host
    enum Snap { kNoSnap, kDevSnap, kHostSnap } snap = kNoSnap;
    size_t snap_off = 0, snap_bytes = 0;
    int64_t snap_n = 0;
    std::vector<uint32_t> snap_host;
    std::deque<Req> q;
    int slot = -1;
    double last_used = 0.0;
    bool failed = false;
    int64_t live = 0;          // live bisectors after its last frame (the export's size)
    bool in_idle = false;      // listed in the server's idle set
    bool in_ready = false;     // listed in the server's ready set
    double idle_key = 0.0;     // its key in the idle set (last use)
    double ready_key = 0.0;    // arrival time of the request it is listed with
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Inst* d_inst = nullptr;
    Counters* d_ctr = nullptr;
    uint32_t* d_map = nullptr;
    Inst* h_inst = nullptr;
    uint32_t* h_map = nullptr;
    Counters* h_ctr = nullptr;
    std::vector<int64_t> ids;
    std::vector<Req> reqs;
    double t_launch = 0.0;
    uint64_t seq = 0;
};

}  // namespace

struct cbt_server_s {
    cbt_server_config cfg{};
    char* arena = nullptr;
    size_t inst_base = 0, inst_bytes = 0, budget = 0, used = 0;
    std::map<size_t, size_t> free_;    // offset -> length, within the instance area
    hipStream_t aux = nullptr;         // admission, eviction and queries
    hipEvent_t aux_done = nullptr;     // the auxiliary stream's work so far (batches wait on it)
    bool aux_pending = false;          // work was queued on it since the last event
    // instances with a queued request and none in flight, by the arrival of
    // their oldest request; resident idle instances (nothing queued or in
    // flight) by last use -- the eviction order
    std::set<std::pair<double, int64_t>> ready, idle;
    // tuned launch schedules by (depth, live count), for instances without a
    // schedule of their own (cbt_server_set_schedule_table)
    struct Sched {
        int32_t D;
        int64_t live;
        int32_t groups, levels;
    };
    std::vector<Sched> sched;
    std::vector<Slot> slots;
    std::unordered_map<int64_t, SInst> inst;
    int64_t next_id = 1;
    uint64_t next_seq = 1;
    std::deque<cbt_completion> done_q;
    cbt_server_stats st{};
};

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool arena_alloc(cbt_server s, size_t bytes, size_t* off)
{
    bytes = round_up(bytes);
    if (s->used + bytes > s->budget) return false;
    for (auto it = s->free_.begin(); it != s->free_.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            s->free_.erase(it);
            if (rest) s->free_[roff] = rest;
            s->used += bytes;
            return true;
        }
    }
    return false;
}

// Snapshots are carved from the top of the highest free range that fits,
// so that workspaces (first fit from the bottom) keep long free ranges.
bool arena_alloc_top(cbt_server s, size_t bytes, size_t* off)
{
    bytes = round_up(bytes);
    if (s->used + bytes > s->budget) return false;
    for (auto it = s->free_.rbegin(); it != s->free_.rend(); ++it) {
        if (it->second >= bytes) {
            const size_t start = it->first, len = it->second;
            *off = start + len - bytes;
            if (len == bytes) s->free_.erase(start);
            else s->free_[start] = len - bytes;
            s->used += bytes;
            return true;
        }
    }
    return false;
}

void arena_free(cbt_server s, size_t off, size_t bytes)
{
    bytes = round_up(bytes);
    s->used -= bytes;
    auto it = s->free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_.erase(nx);
    }
    if (it != s->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_.erase(it);
        }
    }
}

char* inst_ptr(cbt_server s, size_t off) { return s->arena + s->inst_base + off; }

void add_time(double* total, double* longest, double t0)
{
    const double ms = (now_s() - t0) * 1e3;
    *total += ms;
    *longest = ms > *longest ? ms : *longest;
}

// Keeps the instance's entries in the ready set (a queued request, none in
// flight) and the idle set (resident, nothing queued or in flight, not
// failed) in step with its state; called after every change of I.h,
// I.slot, I.q, I.last_used or I.failed.
void refresh_sets(cbt_server s, SInst& I)
{
    if (I.in_idle) {
        s->idle.erase({I.idle_key, I.id});
        I.in_idle = false;
    }
    if (I.h && I.slot < 0 && I.q.empty() && !I.failed) {
        I.idle_key = I.last_used;
        s->idle.insert({I.idle_key, I.id});
        I.in_idle = true;
    }
    if (I.in_ready) {
        s->ready.erase({I.ready_key, I.id});
        I.in_ready = false;
    }
    if (!I.q.empty() && I.slot < 0) {
        I.ready_key = I.q.front().t_arrive;
        s->ready.insert({I.ready_key, I.id});
        I.in_ready = true;
    }
}

// Releases a handle without waiting: every later use of its workspace range
// (an admission's set-up, a snapshot copy) is queued on the same auxiliary
// stream, and an idle instance has no batch in flight.
void release_handle(cbt_handle h)
{
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    cbth::release_counters(h->hctr);
    delete h;
}

// Evicts a resident idle instance: its live records (24 bytes per live
// bisector; their number is known from its last frame) are exported into
// its own vertex cache (48 bytes per block), copied to the arena's top end
// (or to the host when that is full) and the workspace is released.  All on
// the auxiliary stream, which only the host-snapshot path waits for.
cbt_status evict(cbt_server s, SInst& I)
{
    if (!I.h) return CBT_OK;
    const double t0 = now_s();
    cbt_handle h = I.h;
    const cbtk::Pool& P = h->P;
    uint32_t* rec = reinterpret_cast<uint32_t*>(P.vworld);
    const uint32_t n = (uint32_t)I.live;
    HIP_TRY(nullptr, cbtk::launch_enumerate(cbtk::single_launch(P, h->wk, nullptr), s->aux), "enumerate");
    HIP_TRY(nullptr, cbtk::launch_export_live(P, n, rec, s->aux, true), "export live records");
    const size_t bytes = sizeof(uint32_t) * 6 * (size_t)n;
    size_t off = 0;
    if (arena_alloc_top(s, bytes, &off)) {
        HIP_TRY(nullptr, hipMemcpyAsync(inst_ptr(s, off), rec, bytes, hipMemcpyDeviceToDevice, s->aux), "snapshot copy");
        I.snap = SInst::kDevSnap;
        I.snap_off = off;
        I.snap_bytes = bytes;
    } else {
        I.snap_host.resize(6 * (size_t)n);
        HIP_TRY(nullptr, hipMemcpyAsync(I.snap_host.data(), rec, bytes, hipMemcpyDeviceToHost, s->aux), "snapshot copy");
        HIP_TRY(nullptr, hipStreamSynchronize(s->aux), "snapshot copy");
        I.snap = SInst::kHostSnap;
        s->st.host_snapshots++;
    }
    I.snap_n = n;
    release_handle(h);
    I.h = nullptr;
    arena_free(s, I.off, I.bytes);
    s->aux_pending = true;
    s->st.evictions++;
    s->st.resident--;
    s->st.bytes_resident = (int64_t)s->used;
    refresh_sets(s, I);
    add_time(&s->st.evict_ms, &s->st.evict_ms_max, t0);
    return CBT_OK;
}

// Moves an evicted instance's records from the arena to the host.
cbt_status snapshot_to_host(cbt_server s, SInst& I)
{
    I.snap_host.resize(6 * (size_t)I.snap_n);
    HIP_TRY(nullptr, hipMemcpyAsync(I.snap_host.data(), inst_ptr(s, I.snap_off), I.snap_bytes, hipMemcpyDeviceToHost,
                                    s->aux), "snapshot to host");
    HIP_TRY(nullptr, hipStreamSynchronize(s->aux), "snapshot to host");
    arena_free(s, I.snap_off, I.snap_bytes);
    I.snap = SInst::kHostSnap;
    s->st.host_snapshots++;
    s->st.bytes_resident = (int64_t)s->used;
    return CBT_OK;
}

void drop_snapshot(cbt_server s, SInst& I)
{
    if (I.snap == SInst::kDevSnap) arena_free(s, I.snap_off, I.snap_bytes);
    I.snap = SInst::kNoSnap;
    I.snap_n = 0;
    std::vector<uint32_t>().swap(I.snap_host);
    s->st.bytes_resident = (int64_t)s->used;
}

// The state of a handle set up for an import, from live records in device
// memory, queued on the handle's stream without waiting: the pool cleared,
// the records scattered, the bitfield, the sum-reduction tree and the
// vertex cache rebuilt.  A record out of range raises the device error flag,
// which the instance's next frame reports.
cbt_status import_async(cbt_handle h, const uint32_t* records, uint32_t n)
{
    const cbtk::Pool& P = h->P;
    hipStream_t st = h->stream;
    const cbtk::Launch X = cbtk::single_launch(P, h->wk, nullptr);
    HIP_TRY(h, cbtk::launch_clear_pool(P, st), "clear pool");
    HIP_TRY(h, cbtk::launch_import_live(P, n, records, st), "import live records");
    HIP_TRY(h, cbtk::launch_bits_from_ids(P, st), "bitfield");
    HIP_TRY(h, cbtk::launch_reduce(X, st), "sum reduction");
    HIP_TRY(h, cbtk::launch_refresh(X, st, true), "vertex cache");
    h->last_frame_valid = 0;
    return CBT_OK;
}

// Makes I resident: allocates its workspace, initialises it and imports its
// records.  When the budget is exhausted, idle resident instances are
// evicted, least recently used first, then the oldest snapshots in the arena
// move to the host.  CBT_E_BUDGET: cannot fit now.  The set-up of an
// evicted instance from its records in the arena is queued on the auxiliary
// stream without waiting (batches wait for that stream's event); a new
// instance (the base mesh) and records on the host are set up synchronously.
cbt_status admit(cbt_server s, SInst& I, const std::vector<int64_t>& pinned)
{
    if (I.h) return CBT_OK;
    const size_t bytes = cbt_workspace_bytes(I.H, I.D);
    if (!bytes) return cbth::fail(nullptr, CBT_E_DEPTH, "instance %lld: invalid depth", (long long)I.id);
    if (round_up(bytes) > s->budget) {
        I.failed = true;
        refresh_sets(s, I);
        return cbth::fail(nullptr, CBT_E_BUDGET, "instance %lld needs %zu bytes, budget %zu", (long long)I.id, bytes,
                          s->budget);
    }
    size_t off = 0;
    while (!arena_alloc(s, bytes, &off)) {
        SInst* victim = nullptr;
        for (const auto& e : s->idle) {
            SInst& J = s->inst[e.second];
            if (&J == &I || std::find(pinned.begin(), pinned.end(), J.id) != pinned.end()) continue;
            victim = &J;
            break;
        }
        if (victim) {
            cbt_status st = evict(s, *victim);
            if (st) return st;
            continue;
        }
        SInst* old = nullptr;
        for (auto& kv : s->inst) {
            SInst& J = kv.second;
            if (J.snap != SInst::kDevSnap || &J == &I) continue;
            if (!old || J.last_used < old->last_used) old = &J;
        }
        if (!old) return CBT_E_BUDGET;
        cbt_status st = snapshot_to_host(s, *old);
        if (st) return st;
    }
    const double t0 = now_s();
    cbt_mesh m{I.H, I.twin.data(), I.next.data(), I.prev.data(), I.vert.data(), I.V, I.pos.data()};
    cbt_handle h = nullptr;
    // an evicted instance comes back from its live records: the base mesh
    // is not built first (the import clears and fills the pool)
    cbt_status st = I.snap == SInst::kNoSnap
                        ? cbt_init(&m, I.D, inst_ptr(s, off), bytes, s->aux, &h)
                        : cbth::init_for_import(&m, I.D, inst_ptr(s, off), bytes, s->aux, I.roots.data(), &h);
    if (st) {
        arena_free(s, off, bytes);
        I.failed = true;
        refresh_sets(s, I);
        return st;
    }
    if (I.groups) st = cbt_set_schedule(h, I.groups, I.levels);
    if (!st && I.snap != SInst::kNoSnap) {
        // the vertex cache is rebuilt with the instance's own world-position
        // parameters (the camera does not enter them)
        const cbt_camera probe{{0, 0, 1}, {0, 0, -1}, {0, 1, 0}, 1.0f, 16, 16, 1e-3f};
        cbth::make_lodk(&probe, &I.lod, &h->wk);
    }
    if (!st && I.snap == SInst::kDevSnap)
        st = import_async(h, reinterpret_cast<const uint32_t*>(inst_ptr(s, I.snap_off)), (uint32_t)I.snap_n);
    else if (!st && I.snap == SInst::kHostSnap)
        st = cbt_import_live(h, I.snap_host.data(), I.snap_n, 1);
    if (st) {
        cbt_destroy(h);
        arena_free(s, off, bytes);
        I.failed = true;
        refresh_sets(s, I);
        return st;
    }
    I.live = I.snap == SInst::kNoSnap ? I.H : I.snap_n;
    drop_snapshot(s, I);
    I.h = h;
    I.off = off;
    I.bytes = bytes;
    s->aux_pending = true;
    s->st.admissions++;
    s->st.resident++;
    s->st.bytes_resident = (int64_t)s->used;
    refresh_sets(s, I);
    add_time(&s->st.admit_ms, &s->st.admit_ms_max, t0);
    return CBT_OK;
}

void complete(cbt_server s, SInst& I, const Req& r, cbt_status status, const Counters* c, double t_launch,
              int32_t batch_size, double t_done)
{
    cbt_completion o{};
    o.tag = r.tag;
    o.instance = I.id;
    o.status = status;
    o.batch_size = batch_size;
    o.latency_ms = (t_done - r.t_arrive) * 1e3;
    o.queue_ms = (t_launch - r.t_arrive) * 1e3;
    if (c) {
        o.live_before = c->L;
        o.live_after = (int64_t)c->L + c->N - c->stat[cbtk::kStFrees];
    }
    s->done_q.push_back(o);
}

// Completes the queued requests of a failed instance.
void fail_queued(cbt_server s, SInst& I, cbt_status st)
{
    while (!I.q.empty()) {
        complete(s, I, I.q.front(), st, nullptr, now_s(), 0, now_s());
        I.q.pop_front();
    }
    refresh_sets(s, I);
}

// Collects a finished batch.
void harvest(cbt_server s, Slot& S)
{
    const double t = now_s();
    const int32_t n = (int32_t)S.ids.size();
    for (int32_t i = 0; i < n; ++i) {
        auto it = s->inst.find(S.ids[i]);
        if (it == s->inst.end()) continue;
        SInst& I = it->second;
        const Counters& c = S.h_ctr[i];
        cbt_status status = CBT_OK;
        if (c.err) {
            status = CBT_E_DEVICE;
            I.failed = true;
            if (I.h) I.h->failed = 1;
        } else if (I.h) {
            I.h->last_frame_valid = 1;
            I.live = (int64_t)c.L + c.N - c.stat[cbtk::kStFrees];
        }
        I.slot = -1;
        I.last_used = t;
        s->st.frames++;
        s->st.bisector_updates += c.L;
        complete(s, I, S.reqs[i], status, &c, S.t_launch, n, t);
        refresh_sets(s, I);
    }
    S.ids.clear();
    S.reqs.clear();
    S.busy = false;
    s->st.in_flight--;
}

uint64_t grid_need(int32_t D, int32_t groups, int32_t levels);

// The table's schedule for a resident instance: the nearest tuned depth
// (the deeper one on a tie), within it the entry whose live count is
// nearest by ratio to the instance's count after its last frame (its root
// count before the first); taken only when its grids fit the block maps.
void apply_sched(cbt_server s, SInst& I)
{
    int32_t bestD = -1;
    for (const auto& e : s->sched) {
        const int32_t dd = std::abs(e.D - I.D), db = std::abs(bestD - I.D);
        if (bestD < 0 || dd < db || (dd == db && e.D > bestD)) bestD = e.D;
    }
    const double x = std::log((double)std::max<int64_t>(1, I.live > 0 ? I.live : I.H));
    const cbt_server_s::Sched* pick = nullptr;
    double best = 0.0;
    for (const auto& e : s->sched) {
        if (e.D != bestD) continue;
        const double dist = std::fabs(std::log((double)std::max<int64_t>(1, e.live)) - x);
        if (!pick || dist < best) {
            pick = &e;
            best = dist;
        }
    }
    if (!pick || grid_need(I.D, pick->groups, pick->levels) > (uint64_t)s->cfg.map_capacity) return;
    I.h->P.G = (uint32_t)pick->groups;
    I.h->P.sub = pick->levels;
}

cbt_status launch_slot(cbt_server s, Slot& S)
{
    if (s->ready.empty()) return CBT_OK;
    // candidates: the ready set, oldest request first
    std::vector<SInst*> pick;
    std::vector<int64_t> pinned;
    uint64_t nr = 0, nw = 0, nd = 0, nl = 0;
    // Once one admission of this pass has found no memory (after evicting
    // every idle instance it could), the other non-resident candidates wait
    // for a later pass; resident ones are still picked.
    bool no_memory = false;
    for (auto it = s->ready.begin(); it != s->ready.end() && (int32_t)pick.size() < s->cfg.max_batch;) {
        SInst& I = s->inst[it->second];
        ++it;   // I's own entry may be re-inserted below; the next one stays valid
        if (I.failed) {
            fail_queued(s, I, CBT_E_STATE);
            continue;
        }
        if (!I.h && no_memory) continue;
        cbt_status st = admit(s, I, pinned);
        if (st == CBT_E_BUDGET && !I.failed) {   // waits for memory
            no_memory = true;
            continue;
        }
        if (st) {
            fail_queued(s, I, st);
            continue;
        }
        if (!s->sched.empty() && I.groups == 0) apply_sched(s, I);
        const cbtk::Pool& P = I.h->P;
        const uint64_t r = P.G, w = cbtk::word_groups(P), d = cbtk::reduce_groups(P), l = cbtk::list_groups(P);
        if ((nr + r) + (nw + w) + (nd + d) + (nl + l) > (uint64_t)s->cfg.map_capacity) break;
        nr += r;
        nw += w;
        nd += d;
        nl += l;
        pick.push_back(&I);
        pinned.push_back(I.id);
    }
    if (pick.empty()) return CBT_OK;
    const int n = (int)pick.size();
    uint32_t* mr = S.h_map;
    uint32_t* mw = mr + nr;
    uint32_t* md = mw + nw;
    uint32_t* ml = md + nd;
    uint32_t ar = 0, aw = 0, ad = 0, al = 0;
    S.ids.clear();
    S.reqs.clear();
    for (int i = 0; i < n; ++i) {
        SInst& I = *pick[i];
        const Req r = I.q.front();
        I.q.pop_front();
        LodK K;
        cbth::make_lodk(&r.cam, &I.lod, &K);
        cbt_handle h = I.h;
        if (cbth::world_changed(K, h->wk)) {
            h->wk = K;
            HIP_TRY(h, cbtk::launch_refresh(cbtk::single_launch(h->P, K, nullptr), s->aux, false), "vertex cache");
            s->aux_pending = true;
        }
        S.h_inst[i].P = h->P;
        S.h_inst[i].K = K;
        S.h_inst[i].inj = nullptr;
        const uint32_t tag = (uint32_t)i << cbtk::kMapShift;
        for (uint32_t g = 0; g < h->P.G; ++g) mr[ar++] = tag | g;
        for (uint32_t g = 0; g < cbtk::word_groups(h->P); ++g) mw[aw++] = tag | g;
        for (uint32_t g = 0; g < cbtk::reduce_groups(h->P); ++g) md[ad++] = tag | g;
        for (uint32_t g = 0; g < cbtk::list_groups(h->P); ++g) ml[al++] = tag | g;
        I.slot = (int)(&S - s->slots.data());
        refresh_sets(s, I);
        S.ids.push_back(I.id);
        S.reqs.push_back(r);
    }
    cbtk::Launch X{};
    X.batched = true;
    X.B.n = n;
    X.B.inst = S.d_inst;
    X.B.map_rank = S.d_map;
    X.B.map_word = S.d_map + nr;
    X.B.map_red = S.d_map + nr + nw;
    X.B.map_list = S.d_map + nr + nw + nd;
    X.n_inst = (uint32_t)n;
    X.grid_rank = (uint32_t)nr;
    X.grid_word = (uint32_t)nw;
    X.grid_red = (uint32_t)nd;
    X.grid_list = (uint32_t)nl;
    hipStream_t st = S.stream;
    // admissions, evictions and cache refreshes queued on the auxiliary
    // stream come first
    if (s->aux_pending) {
        HIP_TRY(nullptr, hipEventRecord(s->aux_done, s->aux), "auxiliary event");
        s->aux_pending = false;
    }
    HIP_TRY(nullptr, hipStreamWaitEvent(st, s->aux_done, 0), "wait for admissions");
    HIP_TRY(nullptr, hipMemcpyAsync(S.d_inst, S.h_inst, sizeof(Inst) * (size_t)n, hipMemcpyHostToDevice, st), "descriptors");
    HIP_TRY(nullptr, hipMemcpyAsync(S.d_map, S.h_map, 4 * (size_t)(nr + nw + nd + nl), hipMemcpyHostToDevice, st),
            "block maps");
    HIP_TRY(nullptr, cbtk::launch_frame(X, st, nullptr), "batched frame");
    HIP_TRY(nullptr, cbtk::launch_gather_counters(X, S.d_ctr, st), "gather counters");
    HIP_TRY(nullptr, hipMemcpyAsync(S.h_ctr, S.d_ctr, sizeof(Counters) * (size_t)n, hipMemcpyDeviceToHost, st), "counters");
    HIP_TRY(nullptr, hipEventRecord(S.done, st), "batch event");
    S.busy = true;
    S.t_launch = now_s();
    S.seq = s->next_seq++;
    s->st.batches++;
    s->st.in_flight++;
    return CBT_OK;
}

cbt_status progress(cbt_server s)
{
    for (Slot& S : s->slots) {
        if (!S.busy) continue;
        const hipError_t e = hipEventQuery(S.done);
        if (e == hipSuccess) harvest(s, S);
        else if (e != hipErrorNotReady) return cbth::hip_fail(nullptr, e, "batch event");
    }
    for (Slot& S : s->slots) {
        if (S.busy) continue;
        cbt_status st = launch_slot(s, S);
        if (st) return st;
    }
    return CBT_OK;
}

Slot* oldest_busy(cbt_server s)
{
    Slot* o = nullptr;
    for (Slot& S : s->slots)
        if (S.busy && (!o || S.seq < o->seq)) o = &S;
    return o;
}

// workgroups of the four batched grids one instance adds
uint64_t grid_need(int32_t D, int32_t groups, int32_t levels)
{
    cbtk::Pool P{};
    P.D = D;
    P.cap = (uint32_t)(1ull << D);
    P.W = D >= 5 ? (uint32_t)((1ull << D) / 32) : 1u;
    P.G = groups ? (uint32_t)groups : cbth::default_rank_groups(D);
    P.sub = levels ? levels : cbtk::kMaxReduceSub;
    return (uint64_t)P.G + cbtk::word_groups(P) + cbtk::reduce_groups(P) + cbtk::list_groups(P);
}

size_t slot_bytes(const cbt_server_config& c)
{
    return round_up(sizeof(Inst) * (size_t)c.max_batch) + round_up(sizeof(Counters) * (size_t)c.max_batch) +
           round_up(4 * (size_t)c.map_capacity);
}

void destroy_slots(cbt_server s)
{
    for (Slot& S : s->slots) {
        if (S.stream) (void)hipStreamSynchronize(S.stream);
        if (S.done) (void)hipEventDestroy(S.done);
        if (S.stream) (void)hipStreamDestroy(S.stream);
        if (S.h_inst) (void)hipHostFree(S.h_inst);
        if (S.h_map) (void)hipHostFree(S.h_map);
        if (S.h_ctr) (void)hipHostFree(S.h_ctr);
    }
    s->slots.clear();
}

}  // namespace

extern "C" {

size_t cbt_server_overhead_bytes(const cbt_server_config* cfg)
{
    if (!cfg || cfg->max_batch < 1 || cfg->max_batch > cbtk::kMaxBatch || cfg->slots < 1 || cfg->slots > 8 ||
        cfg->map_capacity < 1)
        return 0;
    return slot_bytes(*cfg) * (size_t)cfg->slots;
}

cbt_status cbt_server_create(const cbt_server_config* cfg, void* device_arena, size_t arena_bytes, cbt_server* out)
{
    if (!out) return cbth::fail(nullptr, CBT_E_ARG, "output server pointer is NULL");
    *out = nullptr;
    const size_t over = cbt_server_overhead_bytes(cfg);
    if (!over) return cbth::fail(nullptr, CBT_E_ARG, "invalid server configuration");
    if (!device_arena || (reinterpret_cast<uintptr_t>(device_arena) & (kAlign - 1)))
        return cbth::fail(nullptr, CBT_E_ARG, "device arena must be non-NULL and 256-byte aligned");
    if (arena_bytes < over + kAlign) return cbth::fail(nullptr, CBT_E_BUDGET, "arena smaller than the launch slots (%zu bytes)", over);
    cbt_server s = new (std::nothrow) cbt_server_s();
    if (!s) return cbth::fail(nullptr, CBT_E_ARG, "out of host memory");
    s->cfg = *cfg;
    s->arena = reinterpret_cast<char*>(device_arena);
    s->inst_base = over;
    s->inst_bytes = (arena_bytes - over) & ~(kAlign - 1);
    s->budget = cfg->memory_budget > 0 && (size_t)cfg->memory_budget < s->inst_bytes ? (size_t)cfg->memory_budget
                                                                                      : s->inst_bytes;
    s->free_[0] = s->inst_bytes;
    s->st.bytes_budget = (int64_t)s->budget;
    bool ok = hipStreamCreate(&s->aux) == hipSuccess &&
              hipEventCreateWithFlags(&s->aux_done, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(s->aux_done, s->aux) == hipSuccess;
    s->slots.resize(cfg->slots);
    for (int i = 0; i < cfg->slots && ok; ++i) {
        Slot& S = s->slots[i];
        char* base = s->arena + slot_bytes(*cfg) * (size_t)i;
        S.d_inst = reinterpret_cast<Inst*>(base);
        S.d_ctr = reinterpret_cast<Counters*>(base + round_up(sizeof(Inst) * (size_t)cfg->max_batch));
        S.d_map = reinterpret_cast<uint32_t*>(base + round_up(sizeof(Inst) * (size_t)cfg->max_batch) +
                                              round_up(sizeof(Counters) * (size_t)cfg->max_batch));
        ok = hipStreamCreate(&S.stream) == hipSuccess &&
             hipEventCreateWithFlags(&S.done, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S.h_inst), sizeof(Inst) * (size_t)cfg->max_batch,
                           hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S.h_map), 4 * (size_t)cfg->map_capacity, hipHostMallocDefault) ==
                 hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S.h_ctr), sizeof(Counters) * (size_t)cfg->max_batch,
                           hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        destroy_slots(s);
        if (s->aux_done) (void)hipEventDestroy(s->aux_done);
        if (s->aux) (void)hipStreamDestroy(s->aux);
        delete s;
        return cbth::fail(nullptr, CBT_E_DEVICE, "stream, event or pinned allocation failed");
    }
    *out = s;
    return CBT_OK;
}

cbt_status cbt_server_open(cbt_server s, const cbt_mesh* mesh, int32_t D, const cbt_lod_params* lod,
                           int64_t* instance_id)
{
    if (!s || !mesh || !lod || !instance_id) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    cbt_status st = cbth::validate_mesh(mesh);
    if (st) return st;
    if (!cbt_workspace_bytes(mesh->H, D)) return cbth::fail(nullptr, CBT_E_DEPTH, "invalid H / depth");
    if (grid_need(D, 0, 0) > (uint64_t)s->cfg.map_capacity)
        return cbth::fail(nullptr, CBT_E_ARG, "depth %d needs more workgroups than the map capacity", D);
    cbt_camera probe{{0, 0, 1}, {0, 0, -1}, {0, 1, 0}, 1.0f, 16, 16, 1e-3f};
    st = cbth::check_lod(nullptr, &probe, lod);
    if (st) return st;
    SInst I;
    I.id = s->next_id++;
    I.H = mesh->H;
    I.V = mesh->V;
    I.D = D;
    I.lod = *lod;
    I.twin.assign(mesh->twin, mesh->twin + mesh->H);
    I.next.assign(mesh->next, mesh->next + mesh->H);
    I.prev.assign(mesh->prev, mesh->prev + mesh->H);
    I.vert.assign(mesh->vert, mesh->vert + mesh->H);
    I.pos.assign(mesh->pos, mesh->pos + 3 * (size_t)mesh->V);
    cbth::root_triangles(mesh, I.roots);
    I.last_used = now_s();
    const int64_t id = I.id;
    s->inst.emplace(id, std::move(I));
    s->st.instances++;
    // the mesh is validated now (and the instance admitted when it fits)
    std::vector<int64_t> none;
    st = admit(s, s->inst[id], none);
    if (st && st != CBT_E_BUDGET) {
        s->inst.erase(id);
        s->st.instances--;
        return st;
    }
    if (st == CBT_E_BUDGET && s->inst[id].failed) {
        s->inst.erase(id);
        s->st.instances--;
        return cbth::fail(nullptr, CBT_E_BUDGET, "instance does not fit the memory budget");
    }
    *instance_id = id;
    return CBT_OK;
}

cbt_status cbt_server_set_schedule_table(cbt_server s, int32_t n, const int32_t* depth, const int64_t* live,
                                        const int32_t* rank_groups, const int32_t* reduce_levels)
{
    if (!s) return cbth::fail(nullptr, CBT_E_ARG, "NULL server");
    if (n < 0 || (n > 0 && (!depth || !live || !rank_groups || !reduce_levels)))
        return cbth::fail(nullptr, CBT_E_ARG, "invalid schedule table");
    std::vector<cbt_server_s::Sched> t;
    for (int32_t i = 0; i < n; ++i) {
        if (depth[i] < 0 || depth[i] > 30 || live[i] < 0 || rank_groups[i] < cbtk::kMinRankGroups ||
            rank_groups[i] > cbtk::kMaxRankGroups || reduce_levels[i] < cbtk::kMinReduceSub ||
            reduce_levels[i] > cbtk::kMaxReduceSub)
            return cbth::fail(nullptr, CBT_E_ARG, "schedule table entry %d out of range", i);
        t.push_back({depth[i], live[i], rank_groups[i], reduce_levels[i]});
    }
    s->sched = std::move(t);
    return CBT_OK;
}

cbt_status cbt_server_set_schedule(cbt_server s, int64_t instance_id, int32_t rank_groups, int32_t reduce_levels)
{
    if (!s) return cbth::fail(nullptr, CBT_E_ARG, "NULL server");
    auto it = s->inst.find(instance_id);
    if (it == s->inst.end()) return cbth::fail(nullptr, CBT_E_ARG, "unknown instance %lld", (long long)instance_id);
    SInst& I = it->second;
    if (I.slot >= 0) return cbth::fail(nullptr, CBT_E_STATE, "instance has a request in flight");
    if (grid_need(I.D, rank_groups, reduce_levels) > (uint64_t)s->cfg.map_capacity)
        return cbth::fail(nullptr, CBT_E_ARG, "schedule needs more workgroups than the map capacity");
    if (I.h) {
        cbt_status st = cbt_set_schedule(I.h, rank_groups, reduce_levels);
        if (st) return st;
    } else if (rank_groups < cbtk::kMinRankGroups || rank_groups > cbtk::kMaxRankGroups ||
               reduce_levels < cbtk::kMinReduceSub || reduce_levels > cbtk::kMaxReduceSub) {
        return cbth::fail(nullptr, CBT_E_ARG, "schedule out of range");
    }
    I.groups = rank_groups;
    I.levels = reduce_levels;
    return CBT_OK;
}

cbt_status cbt_server_submit(cbt_server s, int64_t instance_id, const cbt_camera* camera, uint64_t tag)
{
    if (!s || !camera) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    auto it = s->inst.find(instance_id);
    if (it == s->inst.end()) return cbth::fail(nullptr, CBT_E_ARG, "unknown instance %lld", (long long)instance_id);
    SInst& I = it->second;
    if (I.failed) return cbth::fail(nullptr, CBT_E_STATE, "instance %lld failed earlier", (long long)instance_id);
    cbt_status st = cbth::check_lod(nullptr, camera, &I.lod);
    if (st) return st;
    I.q.push_back(Req{tag, *camera, now_s()});
    refresh_sets(s, I);
    s->st.requests++;
    return CBT_OK;
}

cbt_status cbt_server_poll(cbt_server s, int32_t wait, cbt_completion* out, int32_t capacity, int32_t* count)
{
    if (!s || !count || (capacity > 0 && !out) || capacity < 0) return cbth::fail(nullptr, CBT_E_ARG, "invalid argument");
    *count = 0;
    cbt_status st = progress(s);
    if (st) return st;
    if (wait && s->done_q.empty()) {
        Slot* o = oldest_busy(s);
        if (o) {
            HIP_TRY(nullptr, hipEventSynchronize(o->done), "batch wait");
            st = progress(s);
            if (st) return st;
        }
    }
    int32_t n = 0;
    while (n < capacity && !s->done_q.empty()) {
        out[n++] = s->done_q.front();
        s->done_q.pop_front();
    }
    *count = n;
    return CBT_OK;
}

cbt_status cbt_server_drain(cbt_server s)
{
    if (!s) return cbth::fail(nullptr, CBT_E_ARG, "NULL server");
    for (;;) {
        cbt_status st = progress(s);
        if (st) return st;
        Slot* o = oldest_busy(s);
        if (!o) {
            bool queued = false;
            for (auto& kv : s->inst) queued = queued || (!kv.second.q.empty() && !kv.second.failed);
            if (!queued) return CBT_OK;
            // queued requests that cannot be admitted with nothing in flight
            // wait for memory that no completion will free
            bool admissible = false;
            for (auto& kv : s->inst) admissible = admissible || (!kv.second.q.empty() && kv.second.h);
            if (!admissible) return cbth::fail(nullptr, CBT_E_BUDGET, "queued instances do not fit the memory budget");
            continue;
        }
        HIP_TRY(nullptr, hipEventSynchronize(o->done), "batch wait");
    }
}

cbt_status cbt_server_query(cbt_server s, int64_t instance_id, cbt_bisectors* out)
{
    if (!s || !out) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    auto it = s->inst.find(instance_id);
    if (it == s->inst.end()) return cbth::fail(nullptr, CBT_E_ARG, "unknown instance %lld", (long long)instance_id);
    SInst& I = it->second;
    if (I.slot >= 0) {
        Slot& S = s->slots[I.slot];
        HIP_TRY(nullptr, hipEventSynchronize(S.done), "batch wait");
        harvest(s, S);
    }
    if (I.failed) return cbth::fail(nullptr, CBT_E_STATE, "instance %lld failed", (long long)instance_id);
    std::vector<int64_t> none;
    cbt_status st = admit(s, I, none);
    if (st) return st;
    I.last_used = now_s();
    refresh_sets(s, I);
    return cbt_query(I.h, out);   // on the auxiliary stream, after the admission
}

cbt_status cbt_server_close(cbt_server s, int64_t instance_id)
{
    if (!s) return cbth::fail(nullptr, CBT_E_ARG, "NULL server");
    auto it = s->inst.find(instance_id);
    if (it == s->inst.end()) return cbth::fail(nullptr, CBT_E_ARG, "unknown instance %lld", (long long)instance_id);
    SInst& I = it->second;
    if (I.slot >= 0) {
        Slot& S = s->slots[I.slot];
        HIP_TRY(nullptr, hipEventSynchronize(S.done), "batch wait");
        harvest(s, S);
    }
    while (!I.q.empty()) {
        complete(s, I, I.q.front(), CBT_E_STATE, nullptr, now_s(), 0, now_s());
        I.q.pop_front();
    }
    if (I.in_idle) s->idle.erase({I.idle_key, I.id});
    if (I.in_ready) s->ready.erase({I.ready_key, I.id});
    if (I.h) {
        cbt_destroy(I.h);
        arena_free(s, I.off, I.bytes);
        s->st.resident--;
        s->st.bytes_resident = (int64_t)s->used;
    }
    drop_snapshot(s, I);
    s->inst.erase(it);
    s->st.instances--;
    return CBT_OK;
}

cbt_status cbt_server_get_stats(cbt_server s, cbt_server_stats* out)
{
    if (!s || !out) return cbth::fail(nullptr, CBT_E_ARG, "NULL argument");
    int64_t queued = 0;
    for (auto& kv : s->inst) queued += (int64_t)kv.second.q.size();
    *out = s->st;
    out->queued = queued;
    return CBT_OK;
}

cbt_status cbt_server_destroy(cbt_server s)
{
    if (!s) return CBT_OK;
    destroy_slots(s);
    for (auto& kv : s->inst)
        if (kv.second.h) cbt_destroy(kv.second.h);
    if (s->aux) {
        (void)hipStreamSynchronize(s->aux);
        (void)hipStreamDestroy(s->aux);
    }
    if (s->aux_done) (void)hipEventDestroy(s->aux_done);
    delete s;
    return CBT_OK;
}

}  // extern "C"
