/*
 * Sequential CPU reference of the per-frame adaptive bisection update of
 * "Concurrent Binary Trees for Large-Scale Game Components" (Benyoub & Dupuy,
 * 2024).  TEST INFRASTRUCTURE ONLY: this library is loaded by the test suite,
 * by the entry point's smoke check and by the benchmark's CPU-baseline leg,
 * never by the product path.  It shares no code with the HIP library.
 *
 * Everything is plain, single-threaded C99.  Floating point is IEEE binary32,
 * round-to-nearest, built with -ffp-contract=off (no fused multiply-add) so
 * that the same sequence of operations gives the same bits as the GPU.
 *
 * Every function returns 0 on success and a negative code on failure; the
 * message of the last failure is available from orc_last_error().
 */
#ifndef CBT_ORACLE_H
#define CBT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_state orc_state;

/* per-frame counters */
typedef struct {
    int64_t live_before;      /* L, the CBT root before the frame          */
    int64_t free_before;      /* F = 2^D - L                                */
    int64_t split_requests;   /* bisectors whose decision is SPLIT          */
    int64_t split_accepted;   /* initiators that passed the memory budget   */
    int64_t merge_requests;   /* bisectors whose decision is MERGE          */
    int64_t merge_configs;    /* unanimous merge configurations             */
    int64_t merge_accepted;   /* configurations that passed the budget      */
    int64_t merges_executed;  /* configurations merged                      */
    int64_t split_consumed;   /* bisectors consumed by splits (marked)      */
    int64_t allocations;      /* new blocks                                 */
    int64_t frees;            /* released blocks                            */
    int64_t live_after;
    int64_t max_depth;        /* deepest subdivision level after the frame  */
} orc_stats;

/* ---- generic CBT primitives on a full binary heap of 2^(D+1) u32 ---- */
void    orc_cbt_reduce(uint32_t* heap, int32_t D);
int64_t orc_one_to_bit(const uint32_t* heap, int32_t D, int64_t index);
int64_t orc_zero_to_bit(const uint32_t* heap, int32_t D, int64_t index);

/* ---- instance ---- */
orc_state* orc_create(int32_t H, const int32_t* twin, const int32_t* next,
                      const int32_t* prev, const int32_t* vert, int32_t V,
                      const float* pos, int32_t D);
void    orc_destroy(orc_state* s);
int32_t orc_set_lod(orc_state* s, int32_t mode, float split_px, float merge_px,
                    const float* table, int32_t res, float amplitude);
/* size criterion: 0 projected base-edge length (thresholds in pixels, the
 * default), 1 projected triangle area (thresholds in pixels^2), 2 the base
 * edge's length over the distance of its midpoint, in pixels, without
 * frustum culling (cull-free, distance-only) */
int32_t orc_set_criterion(orc_state* s, int32_t criterion);
/* precision of root triangles, decode, world position and the size test:
 * 32 (binary32, the default) or 64 (binary64) */
int32_t orc_set_precision(orc_state* s, int32_t bits);
void    orc_world_position64(const orc_state* s, const double* v, double* p);
int32_t orc_decode64(const orc_state* s, uint64_t id, double* out9);
/* binary64 decode of every live block (9 doubles per block, 0 when free) */
int32_t orc_get_vertices64(const orc_state* s, double* out);
/* camera: float[13] = pos[3], fwd[3], up[3], fovy, width, height, znear.
 * decisions: NULL, or one code per slot (0 keep, 1 split, 2 merge) that
 * replaces the LOD test. */
int32_t orc_frame(orc_state* s, const float* camera, const uint8_t* decisions,
                  orc_stats* stats);

/* ---- inspection ---- */
int32_t orc_depth(const orc_state* s);
int32_t orc_root_bits(const orc_state* s);          /* k = ceil(log2 H) */
int64_t orc_live_count(const orc_state* s);
/* per-slot pool state, arrays of 2^D entries; dead slots read id 0 */
void    orc_get_pool(const orc_state* s, uint64_t* id, int32_t* twin,
                     int32_t* next, int32_t* prev);
void    orc_get_heap(const orc_state* s, uint32_t* heap);  /* 2^(D+1) */
/* flat-domain vertices of every live slot, 9 floats per slot (2^D * 9) */
void    orc_get_vertices(const orc_state* s, float* out);
/* decisions (per slot) and the LOD operands A, Bs, Bm of the last frame */
void    orc_get_decisions(const orc_state* s, uint8_t* dec, float* A,
                          float* Bs, float* Bm);
/* LOD constants derived from a camera: cam[3] right[3] up[3] fwd[3] f2 t2s
 * t2m tx ty znear (18 floats) */
int32_t orc_frame_constants(const orc_state* s, const float* camera, float* out18);
/* world position of a flat-domain point under the instance's LOD mode */
void    orc_world_position(const orc_state* s, const float* v, float* p);
/* flat-domain vertices of the bisector with heap ID id (9 floats) */
int32_t orc_decode(const orc_state* s, uint64_t id, float* out9);
/* root triangle of halfedge h (9 floats) */
void    orc_root_triangle(const orc_state* s, int32_t h, float* out9);
/* replace the whole pool state (live slots given by id != 0) */
int32_t orc_set_pool(orc_state* s, const uint64_t* id, const int32_t* twin,
                     const int32_t* next, const int32_t* prev);
/* structural invariants; 0 when all hold */
int32_t orc_check(const orc_state* s);
/* when nonzero, the literal recursive refinement processes split initiators
 * in the order given by a seeded shuffle instead of rank order (confluence
 * tests); 0 restores rank order */
void    orc_set_initiator_shuffle(orc_state* s, uint64_t seed);
const char* orc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
