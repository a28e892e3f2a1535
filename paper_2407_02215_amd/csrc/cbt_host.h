// Host-only declarations shared by the C-ABI source files: the handle
// behind cbt_handle, status helpers, frame constants.
#pragma once

#include "cbt.h"
#include "cbt_internal.h"

#include <vector>

struct cbt_instance {
    cbtk::Pool P;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    int device;             // HIP device current at initialisation
    int failed;
    int last_frame_valid;   // the live list still describes the last frame
    cbtk::Counters* hctr;   // pinned host mirror of the device counters
    cbtk::LodK wk;          // world-position parameters the vertex cache holds
    int timed_stage;        // stage wrapped by event pairs, 0 = none
    int n_timed;            // event pairs recorded so far
    std::vector<hipEvent_t> events;   // 2 per timed launch
    char err[512];
};

namespace cbth {

cbt_status fail(cbt_handle h, cbt_status st, const char* fmt, ...);
cbt_status hip_fail(cbt_handle h, hipError_t e, const char* what);
cbt_status validate_mesh(const cbt_mesh* m);
// root triangles (Alg. 1) of a validated mesh, 9 floats per halfedge
void root_triangles(const cbt_mesh* m, std::vector<float>& out);
// a binary32 handle on a validated mesh whose pool an import of live
// records (cbt_import_live, same stream) fills next: the root triangles are
// uploaded from roots (kept alive by the caller) and nothing waits
cbt_status init_for_import(const cbt_mesh* mesh, int32_t D, void* device_workspace, size_t workspace_bytes,
                           void* hip_stream, const float* roots, cbt_handle* out);
cbt_status check_lod(cbt_handle h, const cbt_camera* c, const cbt_lod_params* lp);
void make_lodk(const cbt_camera* c, const cbt_lod_params* lp, cbtk::LodK* K);
// the world-position parameters differ from those the vertex cache holds
bool world_changed(const cbtk::LodK& a, const cbtk::LodK& b);
// counters of a finished frame -> cbt_frame_stats (device flags -> CBT_E_DEVICE)
cbt_status stats_from_counters(cbt_handle h, const cbtk::Counters& c, cbt_frame_stats* stats);
uint32_t default_rank_groups(int32_t D);
// a pinned host mirror of one instance's counters (NULL when out of memory)
cbtk::Counters* pinned_counters();
void release_counters(cbtk::Counters* c);

}  // namespace cbth

#define HIP_TRY(h, expr, what)                                   \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return cbth::hip_fail(h, e_, what); \
    } while (0)
