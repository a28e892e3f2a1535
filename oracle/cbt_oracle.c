/*
 * Sequential CPU reference of the per-frame bisection update (see
 * cbt_oracle.h).  TEST INFRASTRUCTURE ONLY -- never linked by the product.
 *
 * Layout of this file, in the order of the paper:
 *   - CBT primitives: sum reduction, OneToBitID (Alg. 7), ZeroToBitID (Alg. 8)
 *     over a binary heap of 2^(D+1) counters (Section 3.1-3.2).
 *   - Instance creation: root bisectors, one per halfedge, in the first H
 *     pool blocks (Section 3.3 "Initialization"), root vertices (Alg. 1).
 *   - Bisector vertices by the splitting matrices M0/M1 (Eq. 1, Alg. 2).
 *   - World position and the screen-space LOD test (Section 3.3 kernel 4,
 *     Section 4.1).
 *   - One frame: the nine pipeline kernels of Section 3.3 executed one after
 *     the other on a single thread.  Splits follow the compatibility chains
 *     of Alg. 3 twice: once as a closure of per-edge split marks (what the
 *     pipeline's command word records) and once literally, recursively, with
 *     the pointer rules of Alg. 5 and Table 1; merges follow Alg. 4 and Alg. 6.
 *     The two split paths must produce the same triangulation.
 *
 * Numbering conventions used throughout:
 *   - heap ID of a bisector: root h has 2^k + h with k = ceil(log2 H); the
 *     children of ID x are 2x and 2x+1 (Section 2.3 "Notation"; Section 3.3
 *     "Initialization", whose printed root index is read as 2^k + h).
 *     depth d = floor(log2 x) - k, root halfedge h = (x >> d) - 2^k.
 *   - the three neighbour pointers name the edges of the vertex triple
 *     (v0, v1, v2): Twin across (v0,v1), Next across (v1,v2), Prev across
 *     (v2,v0).
 */
#include "cbt_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { DEC_KEEP = 0, DEC_SPLIT = 1, DEC_MERGE = 2 };
enum { MARK_B = 1, MARK_N = 2, MARK_P = 4 };   /* split marks: base, Next, Prev edge */
enum { MODE_FLAT = 0, MODE_SPHERE = 1, MODE_HEIGHTFIELD = 2 };
enum { CRIT_EDGE = 0, CRIT_AREA = 1, CRIT_DISTANCE = 2 };   /* projected base-edge length / triangle area /
                                                               base edge over its distance, no culling */

static char g_err[1024];

static int fail(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return -1;
}

const char* orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* CBT primitives (Section 3.1 data layout, Section 3.2 binary searches)      */
/* ------------------------------------------------------------------------ */

/* heap[1] is the root, node i has children 2i and 2i+1, the 2^D leaves
 * heap[2^D + s] hold the bit of block s; every inner node is the sum of its
 * two children. */
void orc_cbt_reduce(uint32_t* heap, int32_t D)
{
    int64_t n = (int64_t)1 << D;
    for (int64_t i = n - 1; i >= 1; --i)
        heap[i] = heap[2 * i] + heap[2 * i + 1];
    heap[0] = 0;
}

/* Alg. 7: index of the index-th bit set to one. */
int64_t orc_one_to_bit(const uint32_t* heap, int32_t D, int64_t index)
{
    int64_t n = (int64_t)1 << D;
    int64_t bit = 1;
    while (bit < n) {
        bit = 2 * bit;
        if (index >= (int64_t)heap[bit]) {
            index -= heap[bit];
            bit += 1;
        }
    }
    return bit - n;
}

/* Alg. 8: index of the index-th bit set to zero; c is the number of leaves
 * below the node being visited. */
int64_t orc_zero_to_bit(const uint32_t* heap, int32_t D, int64_t index)
{
    int64_t n = (int64_t)1 << D;
    int64_t bit = 1;
    int64_t c = n / 2;
    while (bit < n) {
        bit = 2 * bit;
        int64_t zeros = c - (int64_t)heap[bit];
        if (index >= zeros) {
            index -= zeros;
            bit += 1;
        }
        c = c / 2;
    }
    return bit - n;
}

/* ------------------------------------------------------------------------ */
/* instance                                                                  */
/* ------------------------------------------------------------------------ */

struct orc_state {
    int32_t D, k, H, V;
    int64_t cap;
    int32_t *mtwin, *mnext, *mprev, *mvert;
    float* mpos;
    float* root;              /* H * 9 root triangle vertices            */
    uint64_t* id;             /* per slot; 0 = free block                */
    int32_t *twin, *next, *prev;
    uint32_t* heap;           /* 2^(D+1)                                 */
    int32_t mode;
    int32_t criterion;        /* CRIT_EDGE or CRIT_AREA                  */
    int32_t prec;             /* 32 or 64: precision of vertices and LOD  */
    double* root64;           /* H * 9, binary64 variant                 */
    float split_px, merge_px, amp;
    float* table;
    int32_t res;
    uint8_t* dec;
    float *mA, *mBs, *mBm;
    uint64_t shuffle;
};

static int ilog2_u64(uint64_t x)
{
    int r = -1;
    while (x) {
        x >>= 1;
        r++;
    }
    return r;
}

static int depth_of(const orc_state* s, uint64_t id) { return ilog2_u64(id) - s->k; }

/* Alg. 1 with one reading: the average vertex v2 of a face is summed once
 * per face, starting at the face's smallest halfedge index and following
 * Next, so that all root bisectors of a face share bit-identical v2. */
static void compute_root_triangle(const orc_state* s, int32_t h, float* out)
{
    int32_t nx = s->mnext[h];
    const float* a = s->mpos + 3 * s->mvert[h];
    const float* b = s->mpos + 3 * s->mvert[nx];
    int32_t hmin = h;
    for (int32_t g = s->mnext[h]; g != h; g = s->mnext[g])
        if (g < hmin) hmin = g;
    float sum[3];
    for (int c = 0; c < 3; ++c) sum[c] = s->mpos[3 * s->mvert[hmin] + c];
    int n = 1;
    for (int32_t g = s->mnext[hmin]; g != hmin; g = s->mnext[g]) {
        for (int c = 0; c < 3; ++c) sum[c] = sum[c] + s->mpos[3 * s->mvert[g] + c];
        n++;
    }
    for (int c = 0; c < 3; ++c) {
        out[c] = a[c];
        out[3 + c] = b[c];
        out[6 + c] = sum[c] / (float)n;
    }
}

static int validate_mesh(int32_t H, const int32_t* twin, const int32_t* next,
                         const int32_t* prev, const int32_t* vert, int32_t V)
{
    if (H < 3) return fail("mesh needs H >= 3 halfedges (got %d)", H);
    if (V < 1) return fail("mesh needs vertices");
    for (int32_t h = 0; h < H; ++h) {
        if (next[h] < 0 || next[h] >= H || prev[h] < 0 || prev[h] >= H)
            return fail("halfedge %d: next/prev out of range", h);
        if (prev[next[h]] != h || next[prev[h]] != h)
            return fail("halfedge %d: next and prev are not inverse", h);
        if (vert[h] < 0 || vert[h] >= V) return fail("halfedge %d: vertex out of range", h);
        if (twin[h] < -1 || twin[h] >= H || twin[h] == h)
            return fail("halfedge %d: twin out of range", h);
        if (twin[h] >= 0) {
            int32_t t = twin[h];
            if (twin[t] != h) return fail("halfedge %d: twin is not an involution", h);
            if (vert[t] != vert[next[h]] || vert[next[t]] != vert[h])
                return fail("halfedge %d: twin does not run opposite", h);
            if (t == next[h] || t == prev[h]) return fail("halfedge %d: twin inside its own corner", h);
        }
        int32_t n = 1;
        for (int32_t g = next[h]; g != h; g = next[g]) {
            if (++n > H) return fail("halfedge %d: face cycle does not close", h);
        }
        if (n < 3) return fail("halfedge %d: face with fewer than 3 sides", h);
    }
    return 0;
}

orc_state* orc_create(int32_t H, const int32_t* twin, const int32_t* next,
                      const int32_t* prev, const int32_t* vert, int32_t V,
                      const float* pos, int32_t D)
{
    if (!twin || !next || !prev || !vert || !pos) {
        fail("null mesh array");
        return NULL;
    }
    if (validate_mesh(H, twin, next, prev, vert, V)) return NULL;
    int32_t k = 0;
    while (((int64_t)1 << k) < H) k++;
    /* Section 3.3: the pool must hold every root bisector, D >= ceil(log2 H) */
    if (D < k || D < 1 || D > 30) {
        fail("depth D=%d must satisfy ceil(log2 H)=%d <= D <= 30", D, k);
        return NULL;
    }
    orc_state* s = (orc_state*)calloc(1, sizeof *s);
    s->D = D;
    s->k = k;
    s->H = H;
    s->V = V;
    s->cap = (int64_t)1 << D;
    s->mtwin = (int32_t*)malloc(sizeof(int32_t) * H);
    s->mnext = (int32_t*)malloc(sizeof(int32_t) * H);
    s->mprev = (int32_t*)malloc(sizeof(int32_t) * H);
    s->mvert = (int32_t*)malloc(sizeof(int32_t) * H);
    s->mpos = (float*)malloc(sizeof(float) * 3 * V);
    memcpy(s->mtwin, twin, sizeof(int32_t) * H);
    memcpy(s->mnext, next, sizeof(int32_t) * H);
    memcpy(s->mprev, prev, sizeof(int32_t) * H);
    memcpy(s->mvert, vert, sizeof(int32_t) * H);
    memcpy(s->mpos, pos, sizeof(float) * 3 * V);
    s->root = (float*)malloc(sizeof(float) * 9 * H);
    for (int32_t h = 0; h < H; ++h) compute_root_triangle(s, h, s->root + 9 * h);

    s->id = (uint64_t*)calloc(s->cap, sizeof(uint64_t));
    s->twin = (int32_t*)malloc(sizeof(int32_t) * s->cap);
    s->next = (int32_t*)malloc(sizeof(int32_t) * s->cap);
    s->prev = (int32_t*)malloc(sizeof(int32_t) * s->cap);
    s->heap = (uint32_t*)calloc((size_t)2 * s->cap, sizeof(uint32_t));
    s->dec = (uint8_t*)calloc(s->cap, 1);
    s->mA = (float*)calloc(s->cap, sizeof(float));
    s->mBs = (float*)calloc(s->cap, sizeof(float));
    s->mBm = (float*)calloc(s->cap, sizeof(float));
    for (int64_t i = 0; i < s->cap; ++i) s->twin[i] = s->next[i] = s->prev[i] = -1;
    /* Section 3.3 "Initialization": H roots in the first H blocks, their
     * neighbours copied from the halfedge operators, first H bits set, then
     * the sum reduction. */
    for (int32_t h = 0; h < H; ++h) {
        s->id[h] = ((uint64_t)1 << k) + (uint64_t)h;
        s->next[h] = next[h];
        s->prev[h] = prev[h];
        s->twin[h] = twin[h];
        s->heap[s->cap + h] = 1;
    }
    orc_cbt_reduce(s->heap, D);
    s->mode = MODE_FLAT;
    s->prec = 32;
    s->split_px = 8.0f;
    s->merge_px = 4.0f;
    return s;
}

void orc_destroy(orc_state* s)
{
    if (!s) return;
    free(s->mtwin); free(s->mnext); free(s->mprev); free(s->mvert); free(s->mpos);
    free(s->root); free(s->id); free(s->twin); free(s->next); free(s->prev);
    free(s->heap); free(s->dec); free(s->mA); free(s->mBs); free(s->mBm);
    free(s->table); free(s->root64);
    free(s);
}

int32_t orc_set_lod(orc_state* s, int32_t mode, float split_px, float merge_px,
                    const float* table, int32_t res, float amplitude)
{
    if (mode < MODE_FLAT || mode > MODE_HEIGHTFIELD) return fail("unknown LOD mode %d", mode);
    if (mode != MODE_FLAT && (!table || res < 2)) return fail("mode %d needs a table", mode);
    free(s->table);
    s->table = NULL;
    s->res = 0;
    if (mode != MODE_FLAT) {
        size_t n = (size_t)res * res * (mode == MODE_SPHERE ? 6 : 1);
        s->table = (float*)malloc(sizeof(float) * n);
        memcpy(s->table, table, sizeof(float) * n);
        s->res = res;
    }
    s->mode = mode;
    s->split_px = split_px;
    s->merge_px = merge_px;
    s->amp = amplitude;
    return 0;
}

int32_t orc_set_criterion(orc_state* s, int32_t criterion)
{
    if (criterion != CRIT_EDGE && criterion != CRIT_AREA && criterion != CRIT_DISTANCE)
        return fail("unknown size criterion %d", criterion);
    s->criterion = criterion;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* bisector vertices (Eq. 1, Alg. 2)                                         */
/* ------------------------------------------------------------------------ */

/* The subdivision matrix of Alg. 2 is the product of one splitting matrix
 * per level; it is applied here level by level from the root downwards:
 * bit b of the path (most significant first) maps the triple (v0, v1, v2) to
 * M_b (v0, v1, v2), i.e. M0: (v0, v2, m) and M1: (v2, v1, m), m = (v0+v1)/2. */
static void decode_vertices(const orc_state* s, uint64_t id, float* v)
{
    int d = depth_of(s, id);
    int64_t h = (int64_t)(id >> d) - ((int64_t)1 << s->k);
    float v0[3], v1[3], v2[3];
    for (int c = 0; c < 3; ++c) {
        v0[c] = s->root[9 * h + c];
        v1[c] = s->root[9 * h + 3 + c];
        v2[c] = s->root[9 * h + 6 + c];
    }
    for (int i = d - 1; i >= 0; --i) {
        int b = (int)((id >> i) & 1u);
        float m[3];
        for (int c = 0; c < 3; ++c) m[c] = (v0[c] + v1[c]) * 0.5f;
        if (b == 0) {
            for (int c = 0; c < 3; ++c) { v1[c] = v2[c]; v2[c] = m[c]; }
        } else {
            for (int c = 0; c < 3; ++c) { v0[c] = v2[c]; v2[c] = m[c]; }
        }
    }
    for (int c = 0; c < 3; ++c) {
        v[c] = v0[c];
        v[3 + c] = v1[c];
        v[6 + c] = v2[c];
    }
}

/* ------------------------------------------------------------------------ */
/* world position (Section 4.1: vertices are projected on a sphere and      */
/* displaced; terrains are displaced by a height map)                       */
/* ------------------------------------------------------------------------ */

static float bilinear(const float* T, int32_t res, float s, float t)
{
    float fs = floorf(s), ft = floorf(t);
    float lim = (float)(res - 2);
    if (fs < 0.0f) fs = 0.0f;
    if (fs > lim) fs = lim;
    if (ft < 0.0f) ft = 0.0f;
    if (ft > lim) ft = lim;
    int32_t i0 = (int32_t)fs, j0 = (int32_t)ft;
    float fx = s - fs, fy = t - ft;
    float a = T[(int64_t)j0 * res + i0];
    float b = T[(int64_t)j0 * res + i0 + 1];
    float c = T[(int64_t)(j0 + 1) * res + i0];
    float e = T[(int64_t)(j0 + 1) * res + i0 + 1];
    float top = a + fx * (b - a);
    float bot = c + fx * (e - c);
    return top + fy * (bot - top);
}

/* cube-map face = axis of largest magnitude (ties: x, then y, then z),
 * face order +x -x +y -y +z -z, (u, v) = the two other components divided
 * by the magnitude of the major one, in axis order. */
static float sample_cubemap(const orc_state* s, float x, float y, float z)
{
    float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int f;
    float u, v;
    if (ax >= ay && ax >= az) {
        f = x >= 0.0f ? 0 : 1;
        u = y / ax;
        v = z / ax;
    } else if (ay >= az) {
        f = y >= 0.0f ? 2 : 3;
        u = x / ay;
        v = z / ay;
    } else {
        f = z >= 0.0f ? 4 : 5;
        u = x / az;
        v = y / az;
    }
    float hr = 0.5f * (float)(s->res - 1);
    return bilinear(s->table + (int64_t)f * s->res * s->res, s->res, (u + 1.0f) * hr, (v + 1.0f) * hr);
}

static void world_position(const orc_state* s, const float* v, float* p)
{
    if (s->mode == MODE_SPHERE) {
        float len = sqrtf((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        float n0 = v[0] / len, n1 = v[1] / len, n2 = v[2] / len;
        float h = sample_cubemap(s, n0, n1, n2);
        float sc = 1.0f + s->amp * h;
        p[0] = n0 * sc;
        p[1] = n1 * sc;
        p[2] = n2 * sc;
    } else if (s->mode == MODE_HEIGHTFIELD) {
        float r1 = (float)(s->res - 1);
        float h = bilinear(s->table, s->res, v[0] * r1, v[1] * r1);
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2] + s->amp * h;
    } else {
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2];
    }
}

void orc_world_position(const orc_state* s, const float* v, float* p) { world_position(s, v, p); }

/* ------------------------------------------------------------------------ */
/* LOD test (Section 3.3 kernel 4: the decision is taken from the decoded   */
/* vertices and a screen-space size target)                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    float cam[3], right[3], up[3], fwd[3];
    float f2, t2s, t2m, tx, ty, znear;
} lod_consts;

/* camera frame and thresholds, evaluated once per frame in double precision
 * and rounded once to binary32 */
static void make_consts(const orc_state* s, const float* camera, lod_consts* K)
{
    double c[3] = {camera[0], camera[1], camera[2]};
    double f[3] = {camera[3], camera[4], camera[5]};
    double u[3] = {camera[6], camera[7], camera[8]};
    double fovy = camera[9], width = camera[10], height = camera[11], znear = camera[12];
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    double fw[3] = {f[0] / fl, f[1] / fl, f[2] / fl};
    double r[3] = {fw[1] * u[2] - fw[2] * u[1], fw[2] * u[0] - fw[0] * u[2], fw[0] * u[1] - fw[1] * u[0]};
    double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    r[0] /= rl;
    r[1] /= rl;
    r[2] /= rl;
    double up[3] = {r[1] * fw[2] - r[2] * fw[1], r[2] * fw[0] - r[0] * fw[2], r[0] * fw[1] - r[1] * fw[0]};
    double th = tan(0.5 * fovy);
    double focal = 0.5 * height / th;
    for (int i = 0; i < 3; ++i) {
        K->cam[i] = (float)c[i];
        K->right[i] = (float)r[i];
        K->up[i] = (float)up[i];
        K->fwd[i] = (float)fw[i];
    }
    K->f2 = (float)(focal * focal);
    if (s->criterion == CRIT_AREA) {
        /* thresholds are areas in pixels^2; the test compares twice the area */
        K->t2s = (float)(2.0 * (double)s->split_px);
        K->t2m = (float)(2.0 * (double)s->merge_px);
    } else {
        K->t2s = (float)((double)s->split_px * (double)s->split_px);
        K->t2m = (float)((double)s->merge_px * (double)s->merge_px);
    }
    K->tx = (float)(th * width / height);
    K->ty = (float)th;
    K->znear = (float)znear;
}

int32_t orc_frame_constants(const orc_state* s, const float* camera, float* out)
{
    lod_consts K;
    make_consts(s, camera, &K);
    memcpy(out, &K, sizeof K);
    return 0;
}

/* Decision of one bisector.  Reading of the size criterion: the projected
 * length of the refinement (base) edge (v0,v1) in pixels, compared without a
 * division: |proj(v1) - proj(v0)|^2 > tau^2  <=>  A > tau^2 (z0 z1)^2 with
 * A = f^2 ((x1 z0 - x0 z1)^2 + (y1 z0 - y0 z1)^2).  A bisector whose three
 * vertices all lie outside one frustum plane is merged (the triangulation
 * adapts to the view frustum); one whose base edge reaches behind the near
 * plane is split. */
static int classify(const orc_state* s, const lod_consts* K, const float* v,
                    float* oA, float* oBs, float* oBm)
{
    if (s->criterion == CRIT_DISTANCE) {
        /* Cull-free, distance-only variant of the size target (Section 3.3
         * kernel 4 without the frustum adaptation of Section 4.1): the base
         * edge's length e seen face-on from the distance r of its midpoint,
         * f e / r pixels, whatever the view direction.  Compared squared:
         * A = f^2 |p1 - p0|^2 against tau^2 |m - c|^2, m = (p0 + p1) / 2. */
        float p0[3], p1[3];
        world_position(s, v, p0);
        world_position(s, v + 3, p1);
        float mx = (p0[0] + p1[0]) * 0.5f, my = (p0[1] + p1[1]) * 0.5f, mz = (p0[2] + p1[2]) * 0.5f;
        float qx = mx - K->cam[0], qy = my - K->cam[1], qz = mz - K->cam[2];
        float r2 = (qx * qx + qy * qy) + qz * qz;
        float ex = p1[0] - p0[0], ey = p1[1] - p0[1], ez = p1[2] - p0[2];
        float A = K->f2 * ((ex * ex + ey * ey) + ez * ez);
        float Bs = K->t2s * r2;
        float Bm = K->t2m * r2;
        *oA = A;
        *oBs = Bs;
        *oBm = Bm;
        if (A > Bs) return DEC_SPLIT;
        if (A < Bm) return DEC_MERGE;
        return DEC_KEEP;
    }
    float vx[3], vy[3], vz[3];
    for (int i = 0; i < 3; ++i) {
        float p[3];
        world_position(s, v + 3 * i, p);
        float q0 = p[0] - K->cam[0], q1 = p[1] - K->cam[1], q2 = p[2] - K->cam[2];
        vx[i] = (q0 * K->right[0] + q1 * K->right[1]) + q2 * K->right[2];
        vy[i] = (q0 * K->up[0] + q1 * K->up[1]) + q2 * K->up[2];
        vz[i] = (q0 * K->fwd[0] + q1 * K->fwd[1]) + q2 * K->fwd[2];
    }
    int out_near = 1, out_left = 1, out_right = 1, out_bottom = 1, out_top = 1;
    for (int i = 0; i < 3; ++i) {
        float zx = K->tx * vz[i], zy = K->ty * vz[i];
        out_near &= vz[i] < K->znear;
        out_right &= vx[i] > zx;
        out_left &= vx[i] < -zx;
        out_top &= vy[i] > zy;
        out_bottom &= vy[i] < -zy;
    }
    *oA = *oBs = *oBm = 0.0f;
    if (out_near | out_left | out_right | out_bottom | out_top) return DEC_MERGE;
    if (s->criterion == CRIT_AREA) {
        /* The paper's literal target (Section 3.3 kernel 4, Section 4.1): the
         * projected area of the triangle in pixels^2.  With screen
         * coordinates f x_i / z_i, f y_i / z_i, twice the area is
         * f^2 |N| / (z0^2 z1 z2), N = (x1 z0 - x0 z1)(y2 z0 - y0 z2)
         * - (x2 z0 - x0 z2)(y1 z0 - y0 z1), compared without a division.
         * A vertex behind the near plane makes the area unbounded: split. */
        if (vz[0] < K->znear || vz[1] < K->znear || vz[2] < K->znear) return DEC_SPLIT;
        float ax = vx[1] * vz[0] - vx[0] * vz[1];
        float ay = vy[1] * vz[0] - vy[0] * vz[1];
        float bx = vx[2] * vz[0] - vx[0] * vz[2];
        float by = vy[2] * vz[0] - vy[0] * vz[2];
        float N = ax * by - bx * ay;
        float A = K->f2 * fabsf(N);
        float zq = (vz[0] * vz[0]) * (vz[1] * vz[2]);
        float Bs = K->t2s * zq;
        float Bm = K->t2m * zq;
        *oA = A;
        *oBs = Bs;
        *oBm = Bm;
        if (A > Bs) return DEC_SPLIT;
        if (A < Bm) return DEC_MERGE;
        return DEC_KEEP;
    }
    if (vz[0] < K->znear || vz[1] < K->znear) return DEC_SPLIT;
    float ex = vx[1] * vz[0] - vx[0] * vz[1];
    float ey = vy[1] * vz[0] - vy[0] * vz[1];
    float A = K->f2 * (ex * ex + ey * ey);
    float zz = vz[0] * vz[1];
    float z4 = zz * zz;
    float Bs = K->t2s * z4;
    float Bm = K->t2m * z4;
    *oA = A;
    *oBs = Bs;
    *oBm = Bm;
    if (A > Bs) return DEC_SPLIT;
    if (A < Bm) return DEC_MERGE;
    return DEC_KEEP;
}

/* ------------------------------------------------------------------------ */
/* binary64 variant: the paper evaluates its planets' vertex positions in    */
/* double precision (Section 4.2).  The same steps as above -- Alg. 1 roots, */
/* the Eq. 1 / Alg. 2 decode, world position, frame constants (no rounding  */
/* to binary32) and the size test -- in double.                              */
/* ------------------------------------------------------------------------ */

static void compute_root_triangle64(const orc_state* s, int32_t h, double* out)
{
    int32_t nx = s->mnext[h];
    const float* a = s->mpos + 3 * s->mvert[h];
    const float* b = s->mpos + 3 * s->mvert[nx];
    int32_t hmin = h;
    for (int32_t g = s->mnext[h]; g != h; g = s->mnext[g])
        if (g < hmin) hmin = g;
    double sum[3];
    for (int c = 0; c < 3; ++c) sum[c] = s->mpos[3 * s->mvert[hmin] + c];
    int n = 1;
    for (int32_t g = s->mnext[hmin]; g != hmin; g = s->mnext[g]) {
        for (int c = 0; c < 3; ++c) sum[c] = sum[c] + (double)s->mpos[3 * s->mvert[g] + c];
        n++;
    }
    for (int c = 0; c < 3; ++c) {
        out[c] = a[c];
        out[3 + c] = b[c];
        out[6 + c] = sum[c] / (double)n;
    }
}

static void decode_vertices64(const orc_state* s, uint64_t id, double* v)
{
    int d = depth_of(s, id);
    int64_t h = (int64_t)(id >> d) - ((int64_t)1 << s->k);
    double v0[3], v1[3], v2[3];
    for (int c = 0; c < 3; ++c) {
        v0[c] = s->root64[9 * h + c];
        v1[c] = s->root64[9 * h + 3 + c];
        v2[c] = s->root64[9 * h + 6 + c];
    }
    for (int i = d - 1; i >= 0; --i) {
        int b = (int)((id >> i) & 1u);
        double m[3];
        for (int c = 0; c < 3; ++c) m[c] = (v0[c] + v1[c]) * 0.5;
        if (b == 0) {
            for (int c = 0; c < 3; ++c) { v1[c] = v2[c]; v2[c] = m[c]; }
        } else {
            for (int c = 0; c < 3; ++c) { v0[c] = v2[c]; v2[c] = m[c]; }
        }
    }
    for (int c = 0; c < 3; ++c) {
        v[c] = v0[c];
        v[3 + c] = v1[c];
        v[6 + c] = v2[c];
    }
}

static double bilinear64(const float* T, int32_t res, double s, double t)
{
    double fs = floor(s), ft = floor(t);
    double lim = (double)(res - 2);
    if (fs < 0.0) fs = 0.0;
    if (fs > lim) fs = lim;
    if (ft < 0.0) ft = 0.0;
    if (ft > lim) ft = lim;
    int32_t i0 = (int32_t)fs, j0 = (int32_t)ft;
    double fx = s - fs, fy = t - ft;
    double a = T[(int64_t)j0 * res + i0];
    double b = T[(int64_t)j0 * res + i0 + 1];
    double c = T[(int64_t)(j0 + 1) * res + i0];
    double e = T[(int64_t)(j0 + 1) * res + i0 + 1];
    double top = a + fx * (b - a);
    double bot = c + fx * (e - c);
    return top + fy * (bot - top);
}

static double sample_cubemap64(const orc_state* s, double x, double y, double z)
{
    double ax = fabs(x), ay = fabs(y), az = fabs(z);
    int f;
    double u, v;
    if (ax >= ay && ax >= az) {
        f = x >= 0.0 ? 0 : 1;
        u = y / ax;
        v = z / ax;
    } else if (ay >= az) {
        f = y >= 0.0 ? 2 : 3;
        u = x / ay;
        v = z / ay;
    } else {
        f = z >= 0.0 ? 4 : 5;
        u = x / az;
        v = y / az;
    }
    double hr = 0.5 * (double)(s->res - 1);
    return bilinear64(s->table + (int64_t)f * s->res * s->res, s->res, (u + 1.0) * hr, (v + 1.0) * hr);
}

static void world_position64(const orc_state* s, const double* v, double* p)
{
    if (s->mode == MODE_SPHERE) {
        double len = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        double n0 = v[0] / len, n1 = v[1] / len, n2 = v[2] / len;
        double h = sample_cubemap64(s, n0, n1, n2);
        double sc = 1.0 + (double)s->amp * h;
        p[0] = n0 * sc;
        p[1] = n1 * sc;
        p[2] = n2 * sc;
    } else if (s->mode == MODE_HEIGHTFIELD) {
        double r1 = (double)(s->res - 1);
        double h = bilinear64(s->table, s->res, v[0] * r1, v[1] * r1);
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2] + (double)s->amp * h;
    } else {
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2];
    }
}

typedef struct {
    double cam[3], right[3], up[3], fwd[3];
    double f2, t2s, t2m, tx, ty, znear;
} lod_consts64;

static void make_consts64(const orc_state* s, const float* camera, lod_consts64* K)
{
    double f[3] = {camera[3], camera[4], camera[5]};
    double u[3] = {camera[6], camera[7], camera[8]};
    double fovy = camera[9], width = camera[10], height = camera[11];
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    double fw[3] = {f[0] / fl, f[1] / fl, f[2] / fl};
    double r[3] = {fw[1] * u[2] - fw[2] * u[1], fw[2] * u[0] - fw[0] * u[2], fw[0] * u[1] - fw[1] * u[0]};
    double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    r[0] /= rl;
    r[1] /= rl;
    r[2] /= rl;
    double up[3] = {r[1] * fw[2] - r[2] * fw[1], r[2] * fw[0] - r[0] * fw[2], r[0] * fw[1] - r[1] * fw[0]};
    double th = tan(0.5 * fovy);
    double focal = 0.5 * height / th;
    for (int i = 0; i < 3; ++i) {
        K->cam[i] = camera[i];
        K->right[i] = r[i];
        K->up[i] = up[i];
        K->fwd[i] = fw[i];
    }
    K->f2 = focal * focal;
    if (s->criterion == CRIT_AREA) {
        K->t2s = 2.0 * (double)s->split_px;
        K->t2m = 2.0 * (double)s->merge_px;
    } else {
        K->t2s = (double)s->split_px * (double)s->split_px;
        K->t2m = (double)s->merge_px * (double)s->merge_px;
    }
    K->tx = th * width / height;
    K->ty = th;
    K->znear = camera[12];
}

static int classify64(const orc_state* s, const lod_consts64* K, const double* v, float* oA, float* oBs,
                      float* oBm)
{
    if (s->criterion == CRIT_DISTANCE) {   /* as in classify(), in binary64 */
        double p0[3], p1[3];
        world_position64(s, v, p0);
        world_position64(s, v + 3, p1);
        double mx = (p0[0] + p1[0]) * 0.5, my = (p0[1] + p1[1]) * 0.5, mz = (p0[2] + p1[2]) * 0.5;
        double qx = mx - K->cam[0], qy = my - K->cam[1], qz = mz - K->cam[2];
        double r2 = (qx * qx + qy * qy) + qz * qz;
        double ex = p1[0] - p0[0], ey = p1[1] - p0[1], ez = p1[2] - p0[2];
        double A = K->f2 * ((ex * ex + ey * ey) + ez * ez);
        double Bs = K->t2s * r2, Bm = K->t2m * r2;
        *oA = (float)A;
        *oBs = (float)Bs;
        *oBm = (float)Bm;
        if (A > Bs) return DEC_SPLIT;
        if (A < Bm) return DEC_MERGE;
        return DEC_KEEP;
    }
    double vx[3], vy[3], vz[3];
    for (int i = 0; i < 3; ++i) {
        double p[3];
        world_position64(s, v + 3 * i, p);
        double q0 = p[0] - K->cam[0], q1 = p[1] - K->cam[1], q2 = p[2] - K->cam[2];
        vx[i] = (q0 * K->right[0] + q1 * K->right[1]) + q2 * K->right[2];
        vy[i] = (q0 * K->up[0] + q1 * K->up[1]) + q2 * K->up[2];
        vz[i] = (q0 * K->fwd[0] + q1 * K->fwd[1]) + q2 * K->fwd[2];
    }
    int out_near = 1, out_left = 1, out_right = 1, out_bottom = 1, out_top = 1;
    for (int i = 0; i < 3; ++i) {
        double zx = K->tx * vz[i], zy = K->ty * vz[i];
        out_near &= vz[i] < K->znear;
        out_right &= vx[i] > zx;
        out_left &= vx[i] < -zx;
        out_top &= vy[i] > zy;
        out_bottom &= vy[i] < -zy;
    }
    *oA = *oBs = *oBm = 0.0f;
    if (out_near | out_left | out_right | out_bottom | out_top) return DEC_MERGE;
    double A, Bs, Bm;
    if (s->criterion == CRIT_AREA) {
        if (vz[0] < K->znear || vz[1] < K->znear || vz[2] < K->znear) return DEC_SPLIT;
        double ax = vx[1] * vz[0] - vx[0] * vz[1];
        double ay = vy[1] * vz[0] - vy[0] * vz[1];
        double bx = vx[2] * vz[0] - vx[0] * vz[2];
        double by = vy[2] * vz[0] - vy[0] * vz[2];
        double N = ax * by - bx * ay;
        A = K->f2 * fabs(N);
        double zq = (vz[0] * vz[0]) * (vz[1] * vz[2]);
        Bs = K->t2s * zq;
        Bm = K->t2m * zq;
    } else {
        if (vz[0] < K->znear || vz[1] < K->znear) return DEC_SPLIT;
        double ex = vx[1] * vz[0] - vx[0] * vz[1];
        double ey = vy[1] * vz[0] - vy[0] * vz[1];
        A = K->f2 * (ex * ex + ey * ey);
        double zz = vz[0] * vz[1];
        double z4 = zz * zz;
        Bs = K->t2s * z4;
        Bm = K->t2m * z4;
    }
    *oA = (float)A;
    *oBs = (float)Bs;
    *oBm = (float)Bm;
    if (A > Bs) return DEC_SPLIT;
    if (A < Bm) return DEC_MERGE;
    return DEC_KEEP;
}

int32_t orc_set_precision(orc_state* s, int32_t bits)
{
    if (bits != 32 && bits != 64) return fail("precision must be 32 or 64 bits (got %d)", bits);
    if (bits == 64 && !s->root64) {
        s->root64 = (double*)malloc(sizeof(double) * 9 * s->H);
        if (!s->root64) return fail("out of memory");
        for (int32_t h = 0; h < s->H; ++h) compute_root_triangle64(s, h, s->root64 + 9 * h);
    }
    s->prec = bits;
    return 0;
}

void orc_world_position64(const orc_state* s, const double* v, double* p) { world_position64(s, v, p); }

int32_t orc_decode64(const orc_state* s, uint64_t id, double* out9)
{
    if (!s->root64) return fail("binary64 decode needs orc_set_precision(64)");
    int d = depth_of(s, id);
    if (d < 0 || d > 63 - s->k) return fail("ID %llu is not a bisector", (unsigned long long)id);
    int64_t h = (int64_t)(id >> d) - ((int64_t)1 << s->k);
    if (h < 0 || h >= s->H) return fail("ID %llu has no root halfedge", (unsigned long long)id);
    decode_vertices64(s, id, out9);
    return 0;
}

int32_t orc_get_vertices64(const orc_state* s, double* out)
{
    if (!s->root64) return fail("binary64 vertices need orc_set_precision(64)");
    for (int64_t i = 0; i < s->cap; ++i) {
        if (s->id[i]) decode_vertices64(s, s->id[i], out + 9 * i);
        else memset(out + 9 * i, 0, sizeof(double) * 9);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* literal triangulation graph used for Alg. 3-6 and Table 1                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n, cap;
    uint64_t* id;
    int32_t *tw, *nx, *pv;
    uint8_t* leaf;
    int err;
} graph;

static int32_t g_new(graph* g, uint64_t id)
{
    if (g->n == g->cap) {
        g->cap = g->cap * 2 + 64;
        g->id = (uint64_t*)realloc(g->id, sizeof(uint64_t) * g->cap);
        g->tw = (int32_t*)realloc(g->tw, sizeof(int32_t) * g->cap);
        g->nx = (int32_t*)realloc(g->nx, sizeof(int32_t) * g->cap);
        g->pv = (int32_t*)realloc(g->pv, sizeof(int32_t) * g->cap);
        g->leaf = (uint8_t*)realloc(g->leaf, g->cap);
    }
    int32_t x = (int32_t)g->n++;
    g->id[x] = id;
    g->tw[x] = g->nx[x] = g->pv[x] = -1;
    g->leaf[x] = 1;
    return x;
}

/* Alg. 5: the neighbours of a split bisector b now see its children;
 * the Next neighbour borders the second child, the Prev neighbour the first. */
static void refine_pointers(graph* g, int32_t b, int32_t c0, int32_t c1)
{
    int32_t nx = g->nx[b], pv = g->pv[b];
    if (nx >= 0) {
        if (g->pv[nx] == b) g->pv[nx] = c1;
        else if (g->tw[nx] == b) g->tw[nx] = c1;
        else g->err = fail("Alg. 5: Next neighbour of %llu does not point back", (unsigned long long)g->id[b]);
    }
    if (pv >= 0) {
        if (g->nx[pv] == b) g->nx[pv] = c0;
        else if (g->tw[pv] == b) g->tw[pv] = c0;
        else g->err = fail("Alg. 5: Prev neighbour of %llu does not point back", (unsigned long long)g->id[b]);
    }
}

/* split of b (and of its twin k when k >= 0) with the neighbour rules of
 * Table 1, then Alg. 5 for both */
static void split_pair(graph* g, int32_t j, int32_t k)
{
    int32_t c0j = g_new(g, 2 * g->id[j]);
    int32_t c1j = g_new(g, 2 * g->id[j] + 1);
    int32_t c0k = -1, c1k = -1;
    if (k >= 0) {
        c0k = g_new(g, 2 * g->id[k]);
        c1k = g_new(g, 2 * g->id[k] + 1);
    }
    g->nx[c0j] = c1j;
    g->nx[c1j] = c0k;          /* null at a border */
    g->pv[c0j] = c1k;          /* null at a border */
    g->pv[c1j] = c0j;
    g->tw[c0j] = g->pv[j];
    g->tw[c1j] = g->nx[j];
    if (k >= 0) {
        g->nx[c0k] = c1k;
        g->nx[c1k] = c0j;
        g->pv[c0k] = c1j;
        g->pv[c1k] = c0k;
        g->tw[c0k] = g->pv[k];
        g->tw[c1k] = g->nx[k];
    }
    refine_pointers(g, j, c0j, c1j);
    if (k >= 0) refine_pointers(g, k, c0k, c1k);
    g->leaf[j] = 0;
    if (k >= 0) g->leaf[k] = 0;
}

/* Alg. 3.  After the recursive refinement of a coarser twin, the twin of b
 * has become one of that twin's children; it is read again before the pair
 * split. */
static void refine(graph* g, int32_t b, int guard)
{
    if (guard > 200 || g->err) {
        if (!g->err) g->err = fail("Alg. 3: compatibility chain does not terminate");
        return;
    }
    int32_t k = g->tw[b];
    if (k >= 0) {
        if (g->tw[k] != b) {
            refine(g, k, guard + 1);
            k = g->tw[b];
            if (k < 0 || g->tw[k] != b) {
                if (!g->err) g->err = fail("Alg. 3: twin pair not formed for %llu", (unsigned long long)g->id[b]);
                return;
            }
        }
        split_pair(g, b, k);
    } else {
        split_pair(g, b, -1);
    }
}

/* Alg. 6 for one sibling pair (c0 even, c1 odd) merged into a new parent. */
static int32_t merge_pair(graph* g, int32_t c0, int32_t c1)
{
    int32_t p = g_new(g, g->id[c0] >> 1);
    int32_t nx = g->tw[c1], pv = g->tw[c0];
    if (nx >= 0) {
        if (g->pv[nx] == c1) g->pv[nx] = p;
        else if (g->tw[nx] == c1) g->tw[nx] = p;
        else g->err = fail("Alg. 6: neighbour of %llu does not point back", (unsigned long long)g->id[c1]);
    }
    if (pv >= 0) {
        if (g->nx[pv] == c0) g->nx[pv] = p;
        else if (g->tw[pv] == c0) g->tw[pv] = p;
        else g->err = fail("Alg. 6: neighbour of %llu does not point back", (unsigned long long)g->id[c0]);
    }
    /* inverse of Table 1: the parent's Next/Prev edges are the children's
     * base edges */
    g->nx[p] = nx;
    g->pv[p] = pv;
    g->leaf[c0] = 0;
    g->leaf[c1] = 0;
    return p;
}

/* ------------------------------------------------------------------------ */
/* Alg. 4 on the pre-frame pool                                              */
/* ------------------------------------------------------------------------ */

/* Returns the number of members (0 = not mergeable, 2 = border pair,
 * 4 = cycle of four) and writes them to m[] in the order j1, j2, j3, j4. */
static int merge_config(const orc_state* s, int32_t j1, int32_t* m)
{
    uint64_t id1 = s->id[j1];
    if (depth_of(s, id1) < 1) return 0;   /* roots have no parent */
    int bit = (int)(id1 & 1u);
    int32_t j2 = bit ? s->prev[j1] : s->next[j1];
    int32_t j3 = bit ? s->next[j1] : s->prev[j1];
    if (j2 < 0 || (s->id[j2] >> 1) != (id1 >> 1)) return 0;
    m[0] = j1;
    m[1] = j2;
    if (j3 < 0) return 2;
    if (ilog2_u64(s->id[j3]) != ilog2_u64(id1)) return 0;
    int32_t j4 = bit ? s->next[j3] : s->prev[j3];
    if (j4 < 0 || (s->id[j3] >> 1) != (s->id[j4] >> 1)) return 0;
    m[2] = j3;
    m[3] = j4;
    return 4;
}

/* ------------------------------------------------------------------------ */
/* split marks: Alg. 3's compatibility chain as a closure over the edges    */
/* ------------------------------------------------------------------------ */

/* mark(b) records that b's base edge is split; walking through Twin, the
 * chain either ends at a same-level twin pair, at a border, or enters a
 * coarser neighbour through its Next or Prev edge, which that neighbour then
 * splits in addition to its own base edge. */
static int mark_chain(const orc_state* s, uint32_t* marks, int32_t b, int guard)
{
    if (guard > 200) return fail("compatibility chain does not terminate");
    if (marks[b] & MARK_B) return 0;
    marks[b] |= MARK_B;
    int32_t n = s->twin[b];
    if (n < 0) return 0;
    if (s->twin[n] == b) return mark_chain(s, marks, n, guard + 1);
    if (s->next[n] == b) marks[n] |= MARK_N;
    else if (s->prev[n] == b) marks[n] |= MARK_P;
    else return fail("slot %d: twin neighbour %d does not point back", b, n);
    return mark_chain(s, marks, n, guard + 1);
}

/* children created by a mark set, by role: [first child or its two
 * children, second child or its two children]; returns the count and the
 * IDs in ascending order */
static int outputs_of_marks(uint64_t x, uint32_t mk, uint64_t* out)
{
    int n = 0;
    uint64_t c0 = 2 * x, c1 = 2 * x + 1;
    uint64_t tmp[4];
    if (mk & MARK_P) { tmp[n++] = 2 * c0; tmp[n++] = 2 * c0 + 1; }
    else tmp[n++] = c0;
    if (mk & MARK_N) { tmp[n++] = 2 * c1; tmp[n++] = 2 * c1 + 1; }
    else tmp[n++] = c1;
    /* insertion sort, ascending IDs */
    for (int i = 0; i < n; ++i) {
        uint64_t v = tmp[i];
        int j = i - 1;
        while (j >= 0 && out[j] > v) { out[j + 1] = out[j]; j--; }
        out[j + 1] = v;
    }
    return n;
}

typedef struct { uint64_t id; int32_t slot; } id_slot;

static int cmp_id_slot(const void* a, const void* b)
{
    uint64_t x = ((const id_slot*)a)->id, y = ((const id_slot*)b)->id;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int32_t lookup_slot(const id_slot* t, int64_t n, uint64_t id)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (t[mid].id == id) return t[mid].slot;
        if (t[mid].id < id) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static uint64_t splitmix64(uint64_t* x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_set_initiator_shuffle(orc_state* s, uint64_t seed) { s->shuffle = seed; }

/* ------------------------------------------------------------------------ */
/* one frame: the nine kernels of Section 3.3, sequentially                  */
/* ------------------------------------------------------------------------ */

int32_t orc_frame(orc_state* s, const float* camera, const uint8_t* decisions, orc_stats* st)
{
    const int64_t cap = s->cap;
    const int32_t D = s->D;
    const int maxDepth = 63 - s->k;   /* 64-bit IDs */
    int rc = 0;
    orc_stats S;
    memset(&S, 0, sizeof S);

    /* (1) ResetCounter, (2) CachePointers: the live blocks in rank order
     * through Alg. 7; the number of free blocks F bounds all allocations. */
    int64_t L = s->heap[1];
    int64_t F = cap - L;
    S.live_before = L;
    S.free_before = F;
    int32_t* live = (int32_t*)malloc(sizeof(int32_t) * (L > 0 ? L : 1));
    for (int64_t r = 0; r < L; ++r) live[r] = (int32_t)orc_one_to_bit(s->heap, D, r);

    /* (3) ResetCommands */
    uint32_t* marks = (uint32_t*)calloc(cap, sizeof(uint32_t));
    int32_t* cfg_n = (int32_t*)calloc(cap, sizeof(int32_t));
    int32_t* cfg_m = (int32_t*)malloc(sizeof(int32_t) * 4 * cap);
    uint8_t* unanimous = (uint8_t*)calloc(cap, 1);
    uint8_t* merge_acc = (uint8_t*)calloc(cap, 1);
    uint8_t* split_acc = (uint8_t*)calloc(cap, 1);
    uint8_t* merge_exec = (uint8_t*)calloc(cap, 1);
    uint8_t* consumed = (uint8_t*)calloc(cap, 1);
    memset(s->dec, 0, cap);
    memset(s->mA, 0, sizeof(float) * cap);
    memset(s->mBs, 0, sizeof(float) * cap);
    memset(s->mBm, 0, sizeof(float) * cap);

    /* (4) GenerateCommands: decision of every live bisector */
    lod_consts K;
    lod_consts64 K64;
    memset(&K, 0, sizeof K);
    memset(&K64, 0, sizeof K64);
    if (camera) {
        make_consts(s, camera, &K);
        if (s->prec == 64) make_consts64(s, camera, &K64);
    }
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        int d = depth_of(s, s->id[b]);
        int dc;
        if (decisions) {
            dc = decisions[b];
            if (dc > DEC_MERGE) { rc = fail("injected decision %d out of range", dc); goto done; }
        } else if (s->prec == 64) {
            if (!camera) { rc = fail("frame needs a camera or decisions"); goto done; }
            double v[9];
            decode_vertices64(s, s->id[b], v);
            dc = classify64(s, &K64, v, &s->mA[b], &s->mBs[b], &s->mBm[b]);
        } else {
            if (!camera) { rc = fail("frame needs a camera or decisions"); goto done; }
            float v[9];
            decode_vertices(s, s->id[b], v);
            dc = classify(s, &K, v, &s->mA[b], &s->mBs[b], &s->mBm[b]);
        }
        if (dc == DEC_MERGE && d == 0) dc = DEC_KEEP;             /* roots never merge */
        if (dc == DEC_SPLIT && d + 1 > maxDepth) dc = DEC_KEEP;   /* index width limit */
        s->dec[b] = (uint8_t)dc;
        if (dc == DEC_SPLIT) S.split_requests++;
        if (dc == DEC_MERGE) S.merge_requests++;
    }

    /* merge configurations (Alg. 4) and unanimity: every member must itself
     * request a merge and see the same configuration */
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        if (s->dec[b] == DEC_MERGE) cfg_n[b] = merge_config(s, b, cfg_m + 4 * b);
    }
    int64_t Tm = 0;
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        int n = cfg_n[b];
        if (!n) continue;
        int32_t mn = b;
        for (int i = 0; i < n; ++i)
            if (s->id[cfg_m[4 * b + i]] < s->id[mn]) mn = cfg_m[4 * b + i];
        if (mn != b) continue;
        int ok = 1;
        for (int i = 0; i < n && ok; ++i) {
            int32_t m = cfg_m[4 * b + i];
            if (s->dec[m] != DEC_MERGE || cfg_n[m] != n) { ok = 0; break; }
            /* same member set from the member's own view */
            for (int a = 0; a < n; ++a) {
                int found = 0;
                for (int c = 0; c < n; ++c) found |= cfg_m[4 * m + c] == cfg_m[4 * b + a];
                if (!found) {
                    rc = fail("Alg. 4 asymmetric configuration at slot %d", m);
                    goto done;
                }
            }
        }
        if (ok) {
            unanimous[b] = 1;
            Tm += n / 2;        /* one parent per sibling pair */
            S.merge_configs++;
        }
    }

    /* memory budget (reading of the reservation rule): merge reservations
     * first, in rank order, each the exact number of parents, accepted while
     * the running total stays within F; then split reservations of 3d + 4
     * blocks, in rank order, accepted while all merge reservations plus the
     * running split total stay within F. */
    {
        int64_t pm = 0, ps = 0;
        for (int64_t r = 0; r < L; ++r) {
            int32_t b = live[r];
            if (!unanimous[b]) continue;
            pm += cfg_n[b] / 2;
            if (pm <= F) { merge_acc[b] = 1; S.merge_accepted++; }
        }
        for (int64_t r = 0; r < L; ++r) {
            int32_t b = live[r];
            if (s->dec[b] != DEC_SPLIT) continue;
            ps += 3 * depth_of(s, s->id[b]) + 4;
            if (Tm + ps <= F) { split_acc[b] = 1; S.split_accepted++; }
        }
    }

    /* split marks along every accepted compatibility chain */
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        if (split_acc[b] && mark_chain(s, marks, b, 0)) { rc = -1; goto done; }
    }

    /* (5) ReserveBlocks.  A merge executes when its reservation was accepted
     * and no member carries a split mark (splits win).  Owners, in rank
     * order: every marked bisector (2 to 4 children) and the smallest-ID
     * member of every executing merge (1 or 2 parents).  Owner r takes the
     * free blocks ZeroToBitID(P_r + i) of the pre-frame tree, P_r being the
     * number of blocks taken by earlier owners, for its outputs in ascending
     * ID order. */
    int64_t nout_total = 0;
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        if (marks[b]) {
            consumed[b] = 1;
            S.split_consumed++;
        }
    }
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        if (!merge_acc[b]) continue;
        int n = cfg_n[b], clean = 1;
        for (int i = 0; i < n; ++i) clean &= marks[cfg_m[4 * b + i]] == 0;
        if (clean) {
            merge_exec[b] = 1;
            S.merges_executed++;
            for (int i = 0; i < n; ++i) consumed[cfg_m[4 * b + i]] = 1;
        }
    }
    id_slot* outs = (id_slot*)malloc(sizeof(id_slot) * (4 * (size_t)L + 4));
    for (int64_t r = 0; r < L; ++r) {
        int32_t b = live[r];
        uint64_t ids[4];
        int n = 0;
        if (marks[b]) {
            n = outputs_of_marks(s->id[b], marks[b], ids);
        } else if (merge_exec[b]) {
            int cn = cfg_n[b];
            uint64_t p0 = s->id[cfg_m[4 * b + 0]] >> 1;
            if (cn == 2) {
                ids[n++] = p0;
            } else {
                uint64_t p1 = s->id[cfg_m[4 * b + 2]] >> 1;
                ids[n++] = p0 < p1 ? p0 : p1;
                ids[n++] = p0 < p1 ? p1 : p0;
            }
        }
        for (int i = 0; i < n; ++i) {
            if (nout_total >= F) { rc = fail("allocation exceeds the free blocks"); free(outs); goto done; }
            outs[nout_total].id = ids[i];
            outs[nout_total].slot = (int32_t)orc_zero_to_bit(s->heap, D, nout_total);
            nout_total++;
        }
    }
    S.allocations = nout_total;

    /* (6) FillNewBlocks and (7) UpdateNeighbors: the new triangulation is
     * built literally -- Alg. 3 recursion with Table 1 and Alg. 5 for every
     * accepted initiator still unsplit, then Alg. 4 + Alg. 6 for every
     * executing merge -- on a graph whose first nodes are the pool slots. */
    {
        graph g;
        memset(&g, 0, sizeof g);
        g.cap = cap + 64;
        g.id = (uint64_t*)malloc(sizeof(uint64_t) * g.cap);
        g.tw = (int32_t*)malloc(sizeof(int32_t) * g.cap);
        g.nx = (int32_t*)malloc(sizeof(int32_t) * g.cap);
        g.pv = (int32_t*)malloc(sizeof(int32_t) * g.cap);
        g.leaf = (uint8_t*)malloc(g.cap);
        g.n = cap;
        for (int64_t i = 0; i < cap; ++i) {
            g.id[i] = s->id[i];
            g.tw[i] = s->twin[i];
            g.nx[i] = s->next[i];
            g.pv[i] = s->prev[i];
            g.leaf[i] = s->id[i] != 0;
        }
        /* initiator order: rank order, or a seeded permutation */
        int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (L > 0 ? L : 1));
        int64_t ni = 0;
        for (int64_t r = 0; r < L; ++r)
            if (split_acc[live[r]]) order[ni++] = live[r];
        if (s->shuffle) {
            uint64_t st8 = s->shuffle;
            for (int64_t i = ni - 1; i > 0; --i) {
                int64_t j = (int64_t)(splitmix64(&st8) % (uint64_t)(i + 1));
                int32_t t = order[i]; order[i] = order[j]; order[j] = t;
            }
        }
        for (int64_t i = 0; i < ni && !g.err; ++i)
            if (g.leaf[order[i]]) refine(&g, order[i], 0);
        free(order);
        for (int64_t r = 0; r < L && !g.err; ++r) {
            int32_t b = live[r];
            if (!merge_exec[b]) continue;
            int32_t* m = cfg_m + 4 * b;
            int32_t a0 = (s->id[m[0]] & 1) ? m[1] : m[0];
            int32_t a1 = (s->id[m[0]] & 1) ? m[0] : m[1];
            if (cfg_n[b] == 2) {
                int32_t p = merge_pair(&g, a0, a1);
                g.tw[p] = -1;
            } else {
                int32_t q0 = (s->id[m[2]] & 1) ? m[3] : m[2];
                int32_t q1 = (s->id[m[2]] & 1) ? m[2] : m[3];
                int32_t p = merge_pair(&g, a0, a1);
                int32_t q = merge_pair(&g, q0, q1);
                g.tw[p] = q;
                g.tw[q] = p;
            }
        }
        if (g.err) { rc = -1; goto graph_done; }

        /* the two split paths agree: consumed blocks are exactly the graph's
         * interior nodes among the old slots, new leaves exactly the outputs */
        qsort(outs, nout_total, sizeof(id_slot), cmp_id_slot);
        int64_t new_leaves = 0;
        for (int64_t i = 0; i < cap; ++i) {
            if (s->id[i] == 0) continue;
            if (g.leaf[i] == consumed[i]) {
                rc = fail("slot %lld: mark closure and Alg. 3 disagree", (long long)i);
                goto graph_done;
            }
        }
        for (int64_t x = cap; x < g.n; ++x) {
            if (!g.leaf[x]) continue;
            new_leaves++;
            if (lookup_slot(outs, nout_total, g.id[x]) < 0) {
                rc = fail("new bisector %llu of Alg. 3 is not among the reserved outputs",
                          (unsigned long long)g.id[x]);
                goto graph_done;
            }
        }
        if (new_leaves != nout_total) {
            rc = fail("Alg. 3 made %lld new bisectors, reservations %lld", (long long)new_leaves,
                      (long long)nout_total);
            goto graph_done;
        }
        for (int64_t i = 1; i < nout_total; ++i)
            if (outs[i].id == outs[i - 1].id) { rc = fail("duplicate output ID"); goto graph_done; }

        /* slots of the graph's leaves, then the pool write-back */
        int32_t* slot_of = (int32_t*)malloc(sizeof(int32_t) * g.n);
        for (int64_t x = 0; x < g.n; ++x) {
            if (x < cap) slot_of[x] = g.leaf[x] ? (int32_t)x : -1;
            else slot_of[x] = g.leaf[x] ? lookup_slot(outs, nout_total, g.id[x]) : -1;
        }
        for (int64_t i = 0; i < cap; ++i) {
            if (consumed[i]) {
                s->id[i] = 0;
                s->twin[i] = s->next[i] = s->prev[i] = -1;
            }
        }
        for (int64_t x = 0; x < g.n; ++x) {
            if (!g.leaf[x]) continue;
            int32_t sl = slot_of[x];
            int32_t t = g.tw[x], n = g.nx[x], p = g.pv[x];
            if ((t >= 0 && slot_of[t] < 0) || (n >= 0 && slot_of[n] < 0) || (p >= 0 && slot_of[p] < 0)) {
                rc = fail("bisector %llu points to a non-leaf", (unsigned long long)g.id[x]);
                free(slot_of);
                goto graph_done;
            }
            s->id[sl] = g.id[x];
            s->twin[sl] = t >= 0 ? slot_of[t] : -1;
            s->next[sl] = n >= 0 ? slot_of[n] : -1;
            s->prev[sl] = p >= 0 ? slot_of[p] : -1;
        }
        free(slot_of);

        /* (8) UpdateBitfield: release consumed blocks, occupy new ones;
         * (9) SumReduction */
        for (int64_t i = 0; i < cap; ++i)
            if (consumed[i]) { s->heap[cap + i] = 0; S.frees++; }
        for (int64_t i = 0; i < nout_total; ++i) {
            if (s->heap[cap + outs[i].slot]) { rc = fail("allocated block already used"); goto graph_done; }
            s->heap[cap + outs[i].slot] = 1;
        }
        orc_cbt_reduce(s->heap, D);
        S.live_after = s->heap[1];
        int md = 0;
        for (int64_t i = 0; i < cap; ++i)
            if (s->id[i] && depth_of(s, s->id[i]) > md) md = depth_of(s, s->id[i]);
        S.max_depth = md;
    graph_done:
        free(g.id); free(g.tw); free(g.nx); free(g.pv); free(g.leaf);
    }
    free(outs);
done:
    free(live); free(marks); free(cfg_n); free(cfg_m); free(unanimous);
    free(merge_acc); free(split_acc); free(merge_exec); free(consumed);
    if (st) *st = S;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* inspection                                                                */
/* ------------------------------------------------------------------------ */

int32_t orc_depth(const orc_state* s) { return s->D; }
int32_t orc_root_bits(const orc_state* s) { return s->k; }
int64_t orc_live_count(const orc_state* s) { return s->heap[1]; }

void orc_get_pool(const orc_state* s, uint64_t* id, int32_t* twin, int32_t* next, int32_t* prev)
{
    memcpy(id, s->id, sizeof(uint64_t) * s->cap);
    memcpy(twin, s->twin, sizeof(int32_t) * s->cap);
    memcpy(next, s->next, sizeof(int32_t) * s->cap);
    memcpy(prev, s->prev, sizeof(int32_t) * s->cap);
}

void orc_get_heap(const orc_state* s, uint32_t* heap)
{
    memcpy(heap, s->heap, sizeof(uint32_t) * 2 * s->cap);
}

void orc_get_vertices(const orc_state* s, float* out)
{
    for (int64_t i = 0; i < s->cap; ++i) {
        if (s->id[i]) decode_vertices(s, s->id[i], out + 9 * i);
        else memset(out + 9 * i, 0, sizeof(float) * 9);
    }
}

void orc_get_decisions(const orc_state* s, uint8_t* dec, float* A, float* Bs, float* Bm)
{
    if (dec) memcpy(dec, s->dec, s->cap);
    if (A) memcpy(A, s->mA, sizeof(float) * s->cap);
    if (Bs) memcpy(Bs, s->mBs, sizeof(float) * s->cap);
    if (Bm) memcpy(Bm, s->mBm, sizeof(float) * s->cap);
}

int32_t orc_decode(const orc_state* s, uint64_t id, float* out9)
{
    int d = depth_of(s, id);
    if (d < 0 || d > 63 - s->k) return fail("ID %llu is not a bisector", (unsigned long long)id);
    int64_t h = (int64_t)(id >> d) - ((int64_t)1 << s->k);
    if (h < 0 || h >= s->H) return fail("ID %llu has no root halfedge", (unsigned long long)id);
    decode_vertices(s, id, out9);
    return 0;
}

void orc_root_triangle(const orc_state* s, int32_t h, float* out9)
{
    memcpy(out9, s->root + 9 * h, sizeof(float) * 9);
}

int32_t orc_set_pool(orc_state* s, const uint64_t* id, const int32_t* twin,
                     const int32_t* next, const int32_t* prev)
{
    for (int64_t i = 0; i < s->cap; ++i) {
        s->id[i] = id[i];
        s->twin[i] = id[i] ? twin[i] : -1;
        s->next[i] = id[i] ? next[i] : -1;
        s->prev[i] = id[i] ? prev[i] : -1;
        s->heap[s->cap + i] = id[i] != 0;
    }
    orc_cbt_reduce(s->heap, s->D);
    return orc_check(s);
}

/* ------------------------------------------------------------------------ */
/* invariants                                                                */
/* ------------------------------------------------------------------------ */

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int bsearch_u64(const uint64_t* v, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (v[mid] == key) return 1;
        if (v[mid] < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return 0;
}

static void edge_ends(const float* v, int e, const float** a, const float** b)
{
    /* e: 0 = Twin edge (v0,v1), 1 = Next edge (v1,v2), 2 = Prev edge (v2,v0) */
    static const int A[3] = {0, 1, 2}, B[3] = {1, 2, 0};
    *a = v + 3 * A[e];
    *b = v + 3 * B[e];
}

static int same3(const float* a, const float* b) { return memcmp(a, b, 3 * sizeof(float)) == 0; }

int32_t orc_check(const orc_state* s)
{
    const int64_t cap = s->cap;
    /* tree: bits mirror occupancy, inner nodes are sums */
    for (int64_t i = 0; i < cap; ++i)
        if (s->heap[cap + i] != (uint32_t)(s->id[i] != 0)) return fail("bit %lld does not match the pool", (long long)i);
    for (int64_t i = 1; i < cap; ++i)
        if (s->heap[i] != s->heap[2 * i] + s->heap[2 * i + 1]) return fail("tree node %lld is not a sum", (long long)i);
    int64_t L = s->heap[1];
    uint64_t* ids = (uint64_t*)malloc(sizeof(uint64_t) * (L > 0 ? L : 1));
    int64_t n = 0;
    for (int64_t i = 0; i < cap; ++i)
        if (s->id[i]) ids[n++] = s->id[i];
    qsort(ids, n, sizeof(uint64_t), cmp_u64);
    int rc = 0;
    for (int64_t i = 1; i < n && !rc; ++i)
        if (ids[i] == ids[i - 1]) rc = fail("duplicate bisector %llu", (unsigned long long)ids[i]);
    /* complete prefix code per root: no live ancestor, sum of 2^-d is 1 */
    unsigned __int128* area = (unsigned __int128*)calloc(s->H, sizeof(unsigned __int128));
    for (int64_t i = 0; i < n && !rc; ++i) {
        uint64_t x = ids[i];
        int d = depth_of(s, x);
        if (d < 0) { rc = fail("ID %llu below the root level", (unsigned long long)x); break; }
        int64_t h = (int64_t)(x >> d) - ((int64_t)1 << s->k);
        if (h < 0 || h >= s->H) { rc = fail("ID %llu has no root", (unsigned long long)x); break; }
        for (uint64_t a = x >> 1; a && ilog2_u64(a) >= s->k; a >>= 1)
            if (bsearch_u64(ids, n, a)) { rc = fail("%llu and its ancestor %llu are both live", (unsigned long long)x, (unsigned long long)a); break; }
        area[h] += ((unsigned __int128)1) << (100 - d);
    }
    for (int32_t h = 0; h < s->H && !rc; ++h)
        if (area[h] != (((unsigned __int128)1) << 100)) rc = fail("root %d is not exactly covered", h);
    free(area);
    free(ids);
    if (rc) return rc;
    /* pointers: mutual, of an allowed pair type, geometrically shared */
    for (int64_t b = 0; b < cap; ++b) {
        if (!s->id[b]) continue;
        int32_t p3[3] = {s->twin[b], s->next[b], s->prev[b]};
        for (int e = 0; e < 3; ++e)
            for (int f = e + 1; f < 3; ++f)
                if (p3[e] >= 0 && p3[e] == p3[f]) return fail("slot %lld: two pointers to one neighbour", (long long)b);
        float vb[9];
        decode_vertices(s, s->id[b], vb);
        int db = depth_of(s, s->id[b]);
        for (int e = 0; e < 3; ++e) {
            int32_t nb = p3[e];
            if (nb < 0) continue;
            if (nb >= cap || !s->id[nb]) return fail("slot %lld points to a free block", (long long)b);
            int32_t q3[3] = {s->twin[nb], s->next[nb], s->prev[nb]};
            int back = -1, cnt = 0;
            for (int f = 0; f < 3; ++f)
                if (q3[f] == b) { back = f; cnt++; }
            if (cnt != 1) return fail("slot %lld edge %d: neighbour %d does not point back once", (long long)b, e, nb);
            int dn = depth_of(s, s->id[nb]);
            int okt = 0;
            if ((e == 1 && back == 2) || (e == 2 && back == 1) || (e == 0 && back == 0)) okt = dn == db;
            else if (e == 0) okt = db == dn + 1;       /* Twin against Next/Prev */
            else if (back == 0) okt = dn == db + 1;    /* Next/Prev against Twin */
            if (!okt) return fail("slot %lld edge %d: pair type (%d,%d) at depths %d/%d", (long long)b, e, e, back, db, dn);
            float vn[9];
            decode_vertices(s, s->id[nb], vn);
            const float *a0, *a1, *b0, *b1;
            edge_ends(vb, e, &a0, &a1);
            edge_ends(vn, back, &b0, &b1);
            if (!((same3(a0, b0) && same3(a1, b1)) || (same3(a0, b1) && same3(a1, b0))))
                return fail("slot %lld edge %d: shared edge endpoints differ", (long long)b, e);
        }
    }
    return 0;
}
