/*
 * rtsdf_oracle.c -- plain, slow CPU reference of the RTSDF signed-distance hot path
 * (Tan, Chua, Koh, Bhojan, "RTSDF: Real-time Signed Distance Fields for Soft Shadow
 * Approximation in Games", arXiv 2210.06160).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; both are written from the paper.
 *
 * Precision: the paper fixes no precision.  Where floating point decides an integer
 * (a voxel snap, a ray/triangle hit, a rejection-sampling accept) the oracle uses
 * IEEE binary32 with a fixed expression order and no contraction (build with
 * -ffp-contract=off, no fast-math), the same precision the GPU path uses, so the
 * integer outcomes are comparable exactly.  Everything else that is checked by
 * tolerance (BVH culling) is done in binary64.
 *
 * Parity pins live in tests/ (closed forms, brute force, an exact EDT, an independent
 * numpy JFA, rocRAND's Philox).  Every function below is pinned; none is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EMPTY (-1)

typedef struct {
    int32_t nx, ny, nz;
    float org[3];
    float h;
} orc_grid;

static int64_t orc_nvox(orc_grid g) { return (int64_t)g.nx * g.ny * g.nz; }

/* Grid point ids (section 2.2: every grid point may hold "seed information").
 * A seed is identified by the packed coordinates of the voxel it lives in. */
static int32_t orc_pack(int32_t i, int32_t j, int32_t k) { return i | (j << 10) | (k << 20); }
static void orc_unpack(int32_t s, int32_t* i, int32_t* j, int32_t* k)
{
    *i = s & 1023;
    *j = (s >> 10) & 1023;
    *k = (s >> 20) & 1023;
}

int32_t orc_pack_id(int32_t i, int32_t j, int32_t k) { return orc_pack(i, j, k); }

/* ------------------------------------------------------------------------------------
 * Voxelization (section 2.2: "voxelize the scene with voxel resolution equal to our
 * final distance field"; a grid point whose voxel holds a piece of a triangle is a
 * seed).  The paper does not state a method; the reading used here is conservative
 * closed-cell overlap: a voxel is a seed iff the closed cube of the voxel intersects
 * the closed triangle.  Vertices are first snapped to 1/256-voxel fixed point,
 *   X = rint(((v - org) / h) * 256)    (binary32 ops, round-half-even),
 * and the overlap is decided by the separating-axis theorem over the 13 candidate
 * axes of a box and a triangle, in exact 64-bit integers.
 * A triangle with a snapped coordinate beyond +-2^19 (2048 voxels) is not voxelized.
 * ---------------------------------------------------------------------------------- */
#define ORC_SNAP_LIMIT 524288.0f

static int64_t orc_floor_div256(int64_t x)
{
    int64_t q = x / 256;
    if ((x % 256) != 0 && x < 0) q -= 1;
    return q;
}

static int64_t orc_min3(int64_t a, int64_t b, int64_t c)
{
    int64_t m = a < b ? a : b;
    return m < c ? m : c;
}
static int64_t orc_max3(int64_t a, int64_t b, int64_t c)
{
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}
static int64_t orc_abs64(int64_t a) { return a < 0 ? -a : a; }

/* Is the projection of the triangle (three points a[0..2]) onto axis A disjoint from
 * the projection of the box centred at the origin with half-width 128? */
static int orc_axis_separates(const int64_t A[3], int64_t a[3][3])
{
    int64_t p[3];
    for (int v = 0; v < 3; ++v) p[v] = A[0] * a[v][0] + A[1] * a[v][1] + A[2] * a[v][2];
    int64_t r = 128 * (orc_abs64(A[0]) + orc_abs64(A[1]) + orc_abs64(A[2]));
    return orc_min3(p[0], p[1], p[2]) > r || orc_max3(p[0], p[1], p[2]) < -r;
}

static int orc_tri_cell_overlap(int64_t X[3][3], int64_t ci, int64_t cj, int64_t ck)
{
    const int64_t c[3] = {256 * ci + 128, 256 * cj + 128, 256 * ck + 128};
    int64_t a[3][3];
    for (int v = 0; v < 3; ++v)
        for (int d = 0; d < 3; ++d) a[v][d] = X[v][d] - c[d];
    /* the three box face normals */
    for (int d = 0; d < 3; ++d) {
        int64_t e[3] = {0, 0, 0};
        e[d] = 1;
        if (orc_axis_separates(e, a)) return 0;
    }
    /* the triangle's plane normal */
    int64_t f[3][3];
    for (int d = 0; d < 3; ++d) {
        f[0][d] = a[1][d] - a[0][d];
        f[1][d] = a[2][d] - a[1][d];
        f[2][d] = a[0][d] - a[2][d];
    }
    int64_t n[3] = {f[0][1] * f[1][2] - f[0][2] * f[1][1], f[0][2] * f[1][0] - f[0][0] * f[1][2],
                    f[0][0] * f[1][1] - f[0][1] * f[1][0]};
    if (orc_axis_separates(n, a)) return 0;
    /* the nine cross products of triangle edges with box edges */
    for (int m = 0; m < 3; ++m) {
        int64_t ax0[3] = {0, -f[m][2], f[m][1]};
        int64_t ax1[3] = {f[m][2], 0, -f[m][0]};
        int64_t ax2[3] = {-f[m][1], f[m][0], 0};
        if (orc_axis_separates(ax0, a) || orc_axis_separates(ax1, a) || orc_axis_separates(ax2, a))
            return 0;
    }
    return 1;
}

/* Snap one vertex; returns 0 if it is out of the representable range (or not finite). */
static int orc_snap(const float* v, orc_grid g, int64_t X[3])
{
    for (int d = 0; d < 3; ++d) {
        float q = ((v[d] - g.org[d]) / g.h) * 256.0f;
        if (!(fabsf(q) <= ORC_SNAP_LIMIT)) return 0;
        X[d] = (int64_t)rintf(q);
    }
    return 1;
}

/* Returns 0 on success, -1 on a bad triangle index. */
int orc_voxelize(const float* verts, int32_t nv, const int32_t* tris, int32_t nt, orc_grid g,
                 int32_t* seeds)
{
    const int64_t N = orc_nvox(g);
    for (int64_t p = 0; p < N; ++p) seeds[p] = ORC_EMPTY;
    const int32_t dims[3] = {g.nx, g.ny, g.nz};
    for (int32_t t = 0; t < nt; ++t) {
        int64_t X[3][3];
        int ok = 1;
        for (int v = 0; v < 3; ++v) {
            int32_t vi = tris[3 * t + v];
            if (vi < 0 || vi >= nv) return -1;
            if (!orc_snap(verts + 3 * (int64_t)vi, g, X[v])) ok = 0;
        }
        if (!ok) continue;
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = orc_floor_div256(orc_min3(X[0][d], X[1][d], X[2][d]) - 1);
            hi[d] = orc_floor_div256(orc_max3(X[0][d], X[1][d], X[2][d]));
            if (lo[d] < 0) lo[d] = 0;
            if (hi[d] > dims[d] - 1) hi[d] = dims[d] - 1;
            if (lo[d] > hi[d]) ok = 0;
        }
        if (!ok) continue;
        for (int64_t k = lo[2]; k <= hi[2]; ++k)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t i = lo[0]; i <= hi[0]; ++i)
                    if (orc_tri_cell_overlap(X, i, j, k))
                        seeds[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] =
                            orc_pack((int32_t)i, (int32_t)j, (int32_t)k);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Jump flooding (section 2.2).  One pass with offset k: every grid point keeps the seed
 * it already stores and then queries the grid points at p + k*e, e in {-1,0,1}^3 \ {0},
 * in the fixed order ez, ey, ex ascending (-1 < 0 < 1); a queried point that is inside
 * the grid and holds a seed replaces the stored seed only if that seed is strictly
 * closer (squared voxel distance).  Each pass reads only the previous pass's buffer.
 * ---------------------------------------------------------------------------------- */
static int32_t orc_d2(int32_t s, int32_t x, int32_t y, int32_t z)
{
    int32_t sx, sy, sz;
    orc_unpack(s, &sx, &sy, &sz);
    return (sx - x) * (sx - x) + (sy - y) * (sy - y) + (sz - z) * (sz - z);
}

void orc_jfa_pass(const int32_t* in, int32_t* out, orc_grid g, int32_t k)
{
#pragma omp parallel for schedule(static)
    for (int32_t z = 0; z < g.nz; ++z)
        for (int32_t y = 0; y < g.ny; ++y)
            for (int32_t x = 0; x < g.nx; ++x) {
                int64_t p = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
                int32_t best = in[p];
                int32_t bestd2 = best == ORC_EMPTY ? 0 : orc_d2(best, x, y, z);
                for (int ez = -1; ez <= 1; ++ez)
                    for (int ey = -1; ey <= 1; ++ey)
                        for (int ex = -1; ex <= 1; ++ex) {
                            if (ex == 0 && ey == 0 && ez == 0) continue;
                            int32_t qx = x + k * ex, qy = y + k * ey, qz = z + k * ez;
                            if (qx < 0 || qy < 0 || qz < 0 || qx >= g.nx || qy >= g.ny || qz >= g.nz)
                                continue;
                            int32_t s = in[qx + (int64_t)g.nx * (qy + (int64_t)g.ny * qz)];
                            if (s == ORC_EMPTY) continue;
                            int32_t d2 = orc_d2(s, x, y, z);
                            if (best == ORC_EMPTY || d2 < bestd2) {
                                best = s;
                                bestd2 = d2;
                            }
                        }
                out[p] = best;
            }
}

/* Runs the passes in order; the result is left in `seeds`.  `tmp` holds N ints. */
void orc_jfa(int32_t* seeds, int32_t* tmp, orc_grid g, const int32_t* steps, int32_t nsteps)
{
    const int64_t N = orc_nvox(g);
    int32_t* a = seeds;
    int32_t* b = tmp;
    for (int32_t s = 0; s < nsteps; ++s) {
        orc_jfa_pass(a, b, g, steps[s]);
        int32_t* t = a;
        a = b;
        b = t;
    }
    if (a != seeds) memcpy(seeds, a, (size_t)N * sizeof(int32_t));
}

/* Squared voxel distance from each grid point to the seed it stores (-1 if none). */
void orc_seed_d2(const int32_t* seeds, orc_grid g, int32_t* d2)
{
    for (int32_t z = 0; z < g.nz; ++z)
        for (int32_t y = 0; y < g.ny; ++y)
            for (int32_t x = 0; x < g.nx; ++x) {
                int64_t p = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
                d2[p] = seeds[p] == ORC_EMPTY ? -1 : orc_d2(seeds[p], x, y, z);
            }
}

/* ------------------------------------------------------------------------------------
 * Ray mask (section 2.3).  A grid point is ray traced iff the jump-flooded distance is
 * within the mask width; the width is given in voxels, so the test is the exact integer
 * comparison d2 <= band^2 on the stored seed.  The list is in increasing voxel order.
 * Two levels (section 2.3: the coarse field is the mask of a finer traced field; section
 * 2.5.1: coarse 128^3, fine 256^3): with a refinement ratio r the traced grid has r times
 * the points per axis over the same box, fine point (i, j, k) lies in coarse point
 * (i/r, j/r, k/r) (integer division) and is traced iff that coarse point is in the mask;
 * list entries are fine linear indices.  r = 1 is the single-level mask.
 * ---------------------------------------------------------------------------------- */
int64_t orc_band(const int32_t* seeds, orc_grid g, int32_t r, int32_t band, int32_t* list)
{
    int64_t n = 0;
    const int32_t b2 = band * band;
    const int32_t fx = g.nx * r, fy = g.ny * r, fz = g.nz * r;
    for (int32_t z = 0; z < fz; ++z)
        for (int32_t y = 0; y < fy; ++y)
            for (int32_t x = 0; x < fx; ++x) {
                const int32_t cx = x / r, cy = y / r, cz = z / r;
                int32_t s = seeds[cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz)];
                if (s != ORC_EMPTY && orc_d2(s, cx, cy, cz) <= b2) {
                    if (list) list[n] = (int32_t)(x + (int64_t)fx * (y + (int64_t)fy * z));
                    ++n;
                }
            }
    return n;
}

/* ------------------------------------------------------------------------------------
 * Random ray directions (section 2.1: a uniformly distributed point on the unit sphere).
 * Counter-based generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  The counter is
 * (voxel, frame, ray, object<<8 | attempt) and the key is the 64-bit seed.
 * Direction: Marsaglia (1972) -- draw (v1, v2) uniform in [-1,1)^2, reject unless
 * s = v1^2 + v2^2 < 1, then w = (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2 s).
 * Uniforms are u = (word >> 8) * 2^-24 so that v = 2u - 1 is exact in binary32.
 * ---------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

#define ORC_MAX_ATTEMPTS 256

/* Returns the number of Philox calls used (1..256); w = (0,0,1) if all were rejected. */
int orc_direction(uint64_t seed, uint32_t vid, uint32_t frame, uint32_t ray, uint32_t obj, float w[3])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t attempt = 0; attempt < ORC_MAX_ATTEMPTS; ++attempt) {
        const uint32_t ctr[4] = {vid, frame, ray, (obj << 8) | attempt};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        for (int pr = 0; pr < 2; ++pr) {
            float u1 = (float)(r[2 * pr] >> 8) * 0x1p-24f;
            float u2 = (float)(r[2 * pr + 1] >> 8) * 0x1p-24f;
            float v1 = 2.0f * u1 - 1.0f;
            float v2 = 2.0f * u2 - 1.0f;
            float s = v1 * v1 + v2 * v2;
            if (s < 1.0f) {
                float q = sqrtf(1.0f - s);
                w[0] = (2.0f * v1) * q;
                w[1] = (2.0f * v2) * q;
                w[2] = 1.0f - 2.0f * s;
                return (int)attempt + 1;
            }
        }
    }
    w[0] = 0.0f;
    w[1] = 0.0f;
    w[2] = 1.0f;
    return ORC_MAX_ATTEMPTS;
}

/* ------------------------------------------------------------------------------------
 * Ray / triangle hit (section 2.1: minimum traced distance; front or back face from
 * the dot product of the ray direction with the primitive's normal).  Moller & Trumbore
 * (1997) in binary32 with the operation order spelled out below; the geometric normal
 * is (v1-v0) x (v2-v0) with counter-clockwise = outward, so det > 0 <=> dot(w, n) < 0
 * <=> front face.  A hit also requires the computed hit point o + t*w to lie inside the
 * triangle's axis-aligned box widened by `pad` on every side (this only rejects
 * numerically meaningless grazing hits and makes hierarchy culling provably exact).
 * ---------------------------------------------------------------------------------- */
static float orc_dotf(const float a[3], const float b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void orc_crossf(const float a[3], const float b[3], float c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static float orc_min3f(float a, float b, float c)
{
    float m = a < b ? a : b;
    return m < c ? m : c;
}
static float orc_max3f(float a, float b, float c)
{
    float m = a > b ? a : b;
    return m > c ? m : c;
}

int orc_ray_tri(const float o[3], const float w[3], const float v0[3], const float v1[3],
                const float v2[3], float pad, float* t_out, int* front)
{
    float e1[3], e2[3], P[3], T[3], Q[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = v1[d] - v0[d];
        e2[d] = v2[d] - v0[d];
    }
    orc_crossf(w, e2, P);
    float det = orc_dotf(e1, P);
    if (det == 0.0f) return 0;
    float inv = 1.0f / det;
    for (int d = 0; d < 3; ++d) T[d] = o[d] - v0[d];
    float u = orc_dotf(T, P) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return 0;
    orc_crossf(T, e1, Q);
    float v = orc_dotf(w, Q) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return 0;
    float t = orc_dotf(e2, Q) * inv;
    if (!(t > 0.0f)) return 0;
    for (int d = 0; d < 3; ++d) {
        float q = o[d] + t * w[d];
        float lo = orc_min3f(v0[d], v1[d], v2[d]) - pad;
        float hi = orc_max3f(v0[d], v1[d], v2[d]) + pad;
        if (!(q >= lo && q <= hi)) return 0;
    }
    *t_out = t;
    *front = det > 0.0f;
    return 1;
}

/* Closest hit by brute force: lexicographic minimum of (t, triangle index). */
int orc_closest_brute(const float* verts, const int32_t* tris, int32_t nt, const float o[3],
                      const float w[3], float pad, float* t_out, int32_t* tri_out, int* front_out)
{
    int found = 0;
    float bt = INFINITY;
    int32_t btri = -1;
    int bfront = 0;
    for (int32_t t = 0; t < nt; ++t) {
        float th;
        int fr;
        if (orc_ray_tri(o, w, verts + 3 * (int64_t)tris[3 * t], verts + 3 * (int64_t)tris[3 * t + 1],
                        verts + 3 * (int64_t)tris[3 * t + 2], pad, &th, &fr)) {
            if (!found || th < bt) {
                found = 1;
                bt = th;
                btri = t;
                bfront = fr;
            }
        }
    }
    *t_out = bt;
    *tri_out = btri;
    *front_out = bfront;
    return found;
}

/* ------------------------------------------------------------------------------------
 * A plain median-split bounding volume hierarchy, used only to make the oracle fast
 * enough; its closest hit is exactly the brute-force one (tested), because boxes are
 * widened by 2*pad and culled only when the (binary64) slab entry exceeds the best t.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    float lo[3], hi[3];
    int32_t left, right; /* children, or -1 for a leaf */
    int32_t first, count; /* leaf range into the index array */
} orc_node;

typedef struct {
    orc_node* nodes;
    int32_t nnodes;
    int32_t* idx;
    const float* verts;
    const int32_t* tris;
    int32_t nt;
    float pad;
    float* cen; /* centroids, 3 per triangle */
    int sort_axis;
} orc_bvh;

static orc_bvh* g_sort_bvh;
static int orc_cmp_centroid(const void* a, const void* b)
{
    int32_t ia = *(const int32_t*)a, ib = *(const int32_t*)b;
    float ca = g_sort_bvh->cen[3 * ia + g_sort_bvh->sort_axis];
    float cb = g_sort_bvh->cen[3 * ib + g_sort_bvh->sort_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return ia < ib ? -1 : (ia > ib);
}

static int32_t orc_bvh_build_rec(orc_bvh* b, int32_t first, int32_t count)
{
    int32_t me = b->nnodes++;
    orc_node* n = &b->nodes[me];
    for (int d = 0; d < 3; ++d) {
        n->lo[d] = INFINITY;
        n->hi[d] = -INFINITY;
    }
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t q = first; q < first + count; ++q) {
        int32_t t = b->idx[q];
        for (int v = 0; v < 3; ++v) {
            const float* p = b->verts + 3 * (int64_t)b->tris[3 * t + v];
            for (int d = 0; d < 3; ++d) {
                float lo = p[d] - 2.0f * b->pad, hi = p[d] + 2.0f * b->pad;
                if (lo < n->lo[d]) n->lo[d] = lo;
                if (hi > n->hi[d]) n->hi[d] = hi;
            }
        }
        for (int d = 0; d < 3; ++d) {
            float c = b->cen[3 * t + d];
            if (c < clo[d]) clo[d] = c;
            if (c > chi[d]) chi[d] = c;
        }
    }
    n->first = first;
    n->count = count;
    n->left = n->right = -1;
    if (count <= 4) return me;
    int axis = 0;
    float ext = chi[0] - clo[0];
    for (int d = 1; d < 3; ++d)
        if (chi[d] - clo[d] > ext) {
            ext = chi[d] - clo[d];
            axis = d;
        }
    b->sort_axis = axis;
    g_sort_bvh = b;
    qsort(b->idx + first, (size_t)count, sizeof(int32_t), orc_cmp_centroid);
    int32_t half = count / 2;
    int32_t l = orc_bvh_build_rec(b, first, half);
    int32_t r = orc_bvh_build_rec(b, first + half, count - half);
    b->nodes[me].left = l;
    b->nodes[me].right = r;
    return me;
}

void* orc_bvh_build(const float* verts, const int32_t* tris, int32_t nt, float pad)
{
    orc_bvh* b = (orc_bvh*)calloc(1, sizeof(orc_bvh));
    b->verts = verts;
    b->tris = tris;
    b->nt = nt;
    b->pad = pad;
    if (nt == 0) return b;
    b->nodes = (orc_node*)malloc(sizeof(orc_node) * (size_t)(2 * nt));
    b->idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)nt);
    b->cen = (float*)malloc(sizeof(float) * 3 * (size_t)nt);
    for (int32_t t = 0; t < nt; ++t) {
        b->idx[t] = t;
        for (int d = 0; d < 3; ++d) {
            float s = 0.0f;
            for (int v = 0; v < 3; ++v) s += verts[3 * (int64_t)tris[3 * t + v] + d];
            b->cen[3 * t + d] = s / 3.0f;
        }
    }
    orc_bvh_build_rec(b, 0, nt);
    return b;
}

void orc_bvh_free(void* p)
{
    orc_bvh* b = (orc_bvh*)p;
    if (!b) return;
    free(b->nodes);
    free(b->idx);
    free(b->cen);
    free(b);
}

/* Slab test in binary64 against a box; returns 1 and the entry parameter if the ray
 * (t >= 0) meets the box. */
static int orc_slab(const orc_node* n, const float o[3], const float w[3], double* tenter)
{
    double t0 = 0.0, t1 = INFINITY;
    for (int d = 0; d < 3; ++d) {
        if (w[d] == 0.0f) {
            if (o[d] < n->lo[d] || o[d] > n->hi[d]) return 0;
            continue;
        }
        double a = ((double)n->lo[d] - (double)o[d]) / (double)w[d];
        double c = ((double)n->hi[d] - (double)o[d]) / (double)w[d];
        if (a > c) {
            double s = a;
            a = c;
            c = s;
        }
        if (a > t0) t0 = a;
        if (c < t1) t1 = c;
    }
    if (t0 > t1) return 0;
    *tenter = t0;
    return 1;
}

int orc_bvh_closest(const void* bp, const float o[3], const float w[3], float* t_out,
                    int32_t* tri_out, int* front_out)
{
    const orc_bvh* b = (const orc_bvh*)bp;
    float bt = INFINITY;
    int32_t btri = -1;
    int bfront = 0;
    if (b->nt > 0) {
        int32_t stack[256];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const orc_node* n = &b->nodes[stack[--sp]];
            double te;
            if (!orc_slab(n, o, w, &te)) continue;
            if (btri >= 0 && te > (double)bt) continue;
            if (n->left < 0) {
                for (int32_t q = n->first; q < n->first + n->count; ++q) {
                    int32_t t = b->idx[q];
                    float th;
                    int fr;
                    if (orc_ray_tri(o, w, b->verts + 3 * (int64_t)b->tris[3 * t],
                                    b->verts + 3 * (int64_t)b->tris[3 * t + 1],
                                    b->verts + 3 * (int64_t)b->tris[3 * t + 2], b->pad, &th, &fr)) {
                        if (btri < 0 || th < bt || (th == bt && t < btri)) {
                            bt = th;
                            btri = t;
                            bfront = fr;
                        }
                    }
                }
            } else {
                stack[sp++] = n->right;
                stack[sp++] = n->left;
            }
        }
    }
    *t_out = bt;
    *tri_out = btri;
    *front_out = bfront;
    return btri >= 0;
}

/* ------------------------------------------------------------------------------------
 * Ray sampling of listed grid points (section 2.1).  For each listed voxel, ray j of
 * this frame starts at the voxel centre org + h*(i + 0.5) and goes along the Philox /
 * Marsaglia direction.  Every ray that hits counts one front or one back hit (front in
 * the low 16 bits, back in the high 16 bits), lowers the stored minimum distance, and
 * lowers the 64-bit record  bits(t) << 32 | (frame * x + j)  that names the ray which
 * produced the minimum.  Outputs are indexed like the list and are accumulated into.
 * ---------------------------------------------------------------------------------- */
void orc_voxel_centre(orc_grid g, int64_t vid, float o[3])
{
    int64_t i = vid % g.nx, j = (vid / g.nx) % g.ny, k = vid / ((int64_t)g.nx * g.ny);
    o[0] = g.org[0] + g.h * ((float)i + 0.5f);
    o[1] = g.org[1] + g.h * ((float)j + 0.5f);
    o[2] = g.org[2] + g.h * ((float)k + 0.5f);
}

void orc_raysample(const void* bvh, orc_grid g, const int32_t* vids, int64_t n, int32_t x,
                   uint64_t seed, uint32_t frame, uint32_t obj, float* dmin, uint32_t* hits,
                   uint64_t* argmin)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; ++q) {
        float o[3];
        orc_voxel_centre(g, vids[q], o);
        for (int32_t j = 0; j < x; ++j) {
            float w[3], t;
            int32_t tri;
            int fr;
            orc_direction(seed, (uint32_t)vids[q], frame, (uint32_t)j, obj, w);
            if (!orc_bvh_closest(bvh, o, w, &t, &tri, &fr)) continue;
            if (t < dmin[q]) dmin[q] = t;
            hits[q] += fr ? 1u : 65536u;
            uint32_t tb;
            memcpy(&tb, &t, 4);
            uint64_t rec = ((uint64_t)tb << 32) | (uint64_t)(frame * (uint32_t)x + (uint32_t)j);
            if (argmin && rec < argmin[q]) argmin[q] = rec;
        }
    }
}

/* ------------------------------------------------------------------------------------
 * Combining the coarse and the ray-traced field.
 *   coarse magnitude  u = h * sqrt(d2)   (binary32, correctly rounded sqrt; +inf if no seed)
 *   coarse SDF        c = u - beta       (section 2.2: subtract a small beta for a sign)
 *   in band           d2 <= band^2       (section 2.3)
 *   sign              negative iff back hits > front hits (section 2.1)
 * mode 0, running minimum (section 2.1): in band with at least one hit the value is
 *   +-dmin, otherwise c.
 * mode 1, decay (section 2.5.1, Eq. 1) on magnitudes: in band
 *   m_t = min(alpha * m_{t-1} + (1 - alpha) * u_t, r_t), r_t = this frame's dmin or
 *   +inf without hits; the sign is this frame's majority, or the previous sign on a tie;
 *   state = sign * m_t.  Outside the band state = +u_t.  `reset` (or a non-finite
 *   previous state) starts from m_{-1} = u_t with a positive sign.
 * Both modes then subtract `bias` (section 2.5.3: thicken surfaces).
 * The voxels combined are vids[0..n) (all voxels if vids is NULL); the outputs dmin,
 * hits, state and fine are indexed like vids.
 * ---------------------------------------------------------------------------------- */
void orc_combine(const int32_t* seeds, const float* dmin, const uint32_t* hits, orc_grid g, int32_t r,
                 const int32_t* vids, int64_t n, int32_t band, float beta, float bias, int32_t mode,
                 float alpha, int32_t reset, float* state, float* fine)
{
    /* g is the jump-flooded grid; the combined field has r times its points per axis and
     * each of its points takes the coarse distance of the coarse point it lies in */
    const float oma = 1.0f - alpha;
    const int64_t fx = (int64_t)g.nx * r, fy = (int64_t)g.ny * r;
    if (!vids) n = orc_nvox(g) * r * r * r;
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = vids ? vids[q] : q;
        int32_t x = (int32_t)((p % fx) / r), y = (int32_t)(((p / fx) % fy) / r),
                z = (int32_t)((p / (fx * fy)) / r);
        int32_t s = seeds[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)];
        float u;
        int inband;
        if (s == ORC_EMPTY) {
            u = INFINITY;
            inband = 0;
        } else {
            int32_t d2 = orc_d2(s, x, y, z);
            u = g.h * sqrtf((float)d2);
            inband = d2 <= band * band;
        }
        float c = u - beta;
        uint32_t front = hits[q] & 0xFFFFu, back = hits[q] >> 16;
        float val;
        if (mode == 0) {
            if (inband && (front + back) > 0)
                val = back > front ? -dmin[q] : dmin[q];
            else
                val = c;
        } else {
            if (!inband) {
                state[q] = u;
                val = c;
            } else {
                float prev = state[q];
                float mprev, sprev;
                if (reset || !isfinite(prev)) {
                    mprev = u;
                    sprev = 1.0f;
                } else {
                    mprev = fabsf(prev);
                    sprev = signbit(prev) ? -1.0f : 1.0f;
                }
                float blend = alpha * mprev + oma * u;
                float r = (front + back) > 0 ? dmin[q] : INFINITY;
                float m = blend < r ? blend : r;
                float sg = back > front ? -1.0f : (front > back ? 1.0f : sprev);
                state[q] = copysignf(m, sg);
                val = state[q];
            }
        }
        fine[q] = val - bias;
    }
}

/* ------------------------------------------------------------------------------------
 * Soft shadows by sphere tracing the fine field (section 2.4).  The paper prints no
 * formula; the reading used: from a receiver point P march towards the light along the
 * unit direction l, starting at t = t0 (at least one voxel, section 2.5.3), for a fixed
 * number of steps; each step samples s = trilinear(fine, P + t l), keeps
 * res = min(res, k s / t) (penumbra estimate of the closest approach, section 2.4) and
 * advances t by s clamped to [smin, smax] (section 2.5.2 caps the step at 0.05).  The
 * pixel value is clamp(res, 0, 1) with res starting at 1.  Binary64 throughout.
 * Trilinear sampling: grid coordinate g = (X - org)/h - 1/2 (voxel centres are integers),
 * clamped to [0, n-1]; i0 = min(floor(g), n-2); f = g - i0; interpolate in x, then y, then
 * z with a + f (b - a).
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t width, height;  /* pixel (a, b): P = (x0 + (a+1/2) dx, y, z0 + (b+1/2) dz); img[b*width + a] */
    float x0, z0, dx, dz, y;
    float light[3];          /* unit direction towards the light */
    float k;                 /* penumbra sharpness */
    int32_t steps;
    float smin, smax, t0;
} orc_shadow;

static double orc_fetch(const double* f, orc_grid g, int64_t i, int64_t j, int64_t k)
{
    return f[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)];
}

/* value and gradient (with respect to the world position) of the trilinear interpolant */
static double orc_trilinear(const double* f, orc_grid g, const double X[3], double grad[3])
{
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    int64_t i0[3];
    double fr[3];
    int inside[3];
    for (int a = 0; a < 3; ++a) {
        double c = (X[a] - (double)g.org[a]) / (double)g.h - 0.5;
        inside[a] = c > 0.0 && c < (double)(n[a] - 1);
        if (c < 0.0) c = 0.0;
        if (c > (double)(n[a] - 1)) c = (double)(n[a] - 1);
        int64_t b = (int64_t)floor(c);
        if (b > n[a] - 2) b = n[a] - 2;
        if (b < 0) b = 0;
        i0[a] = b;
        fr[a] = n[a] > 1 ? c - (double)b : 0.0;
    }
    const int64_t i1[3] = {n[0] > 1 ? i0[0] + 1 : i0[0], n[1] > 1 ? i0[1] + 1 : i0[1], n[2] > 1 ? i0[2] + 1 : i0[2]};
    double c[2][2][2];
    for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
            for (int x = 0; x < 2; ++x)
                c[z][y][x] = orc_fetch(f, g, x ? i1[0] : i0[0], y ? i1[1] : i0[1], z ? i1[2] : i0[2]);
    double cx[2][2], dcx[2][2];
    for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y) {
            cx[z][y] = c[z][y][0] + fr[0] * (c[z][y][1] - c[z][y][0]);
            dcx[z][y] = c[z][y][1] - c[z][y][0];
        }
    double cy[2], dcyx[2], dcyy[2];
    for (int z = 0; z < 2; ++z) {
        cy[z] = cx[z][0] + fr[1] * (cx[z][1] - cx[z][0]);
        dcyx[z] = dcx[z][0] + fr[1] * (dcx[z][1] - dcx[z][0]);
        dcyy[z] = cx[z][1] - cx[z][0];
    }
    const double v = cy[0] + fr[2] * (cy[1] - cy[0]);
    if (grad) {
        grad[0] = inside[0] ? (dcyx[0] + fr[2] * (dcyx[1] - dcyx[0])) / (double)g.h : 0.0;
        grad[1] = inside[1] ? (dcyy[0] + fr[2] * (dcyy[1] - dcyy[0])) / (double)g.h : 0.0;
        grad[2] = inside[2] ? (cy[1] - cy[0]) / (double)g.h : 0.0;
    }
    return v;
}

/* adds w * d(value)/d(corner values) into gf */
static void orc_trilinear_scatter(double* gf, orc_grid g, const double X[3], double w)
{
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    int64_t i0[3], i1[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double c = (X[a] - (double)g.org[a]) / (double)g.h - 0.5;
        if (c < 0.0) c = 0.0;
        if (c > (double)(n[a] - 1)) c = (double)(n[a] - 1);
        int64_t b = (int64_t)floor(c);
        if (b > n[a] - 2) b = n[a] - 2;
        if (b < 0) b = 0;
        i0[a] = b;
        i1[a] = n[a] > 1 ? b + 1 : b;
        fr[a] = n[a] > 1 ? c - (double)b : 0.0;
    }
    for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
            for (int x = 0; x < 2; ++x) {
                const double wt = (x ? fr[0] : 1.0 - fr[0]) * (y ? fr[1] : 1.0 - fr[1]) * (z ? fr[2] : 1.0 - fr[2]);
                gf[(x ? i1[0] : i0[0]) + (int64_t)g.nx * ((y ? i1[1] : i0[1]) + (int64_t)g.ny * (z ? i1[2] : i0[2]))] +=
                    w * wt;
            }
}

/* trilinear value and positional gradient at n points X[3 n] (for tests) */
void orc_sample(const double* fine, orc_grid g, const double* X, int64_t n, double* val, double* grad)
{
    for (int64_t q = 0; q < n; ++q) val[q] = orc_trilinear(fine, g, X + 3 * q, grad ? grad + 3 * q : NULL);
}

static void orc_pixel_origin(const orc_shadow* s, int32_t a, int32_t b, double P[3])
{
    P[0] = (double)s->x0 + ((double)a + 0.5) * (double)s->dx;
    P[1] = (double)s->y;
    P[2] = (double)s->z0 + ((double)b + 0.5) * (double)s->dz;
}

/* ------------------------------------------------------------------------------------
 * Two-sample triangulation of the closest approach (section 2.5.2, after Aaltonen 2018).
 * The paper prints no formula; the reading used: consecutive samples s_{m-1} = r1 at
 * P + t_{m-1} l and s_m = r2 at P + t_m l each bound an empty sphere; the step between
 * them is delta = clamp(r1, smin, smax).  The two sphere surfaces meet on a circle in the
 * plane perpendicular to the ray at distance y = (r2^2 - r1^2 + delta^2) / (2 delta)
 * behind the later sample, with radius d = sqrt(r2^2 - y^2): the nearest point to the ray
 * that both samples allow.  The estimate at step m is k d / (t_m - y) when r1 > 0, r2 > 0,
 * d^2 > 0 and t_m - y > 0, else the one-sample k r2 / t_m.  (For a point occluder both
 * spheres pass through the point, so d is exactly its distance from the ray.)  Binary64.
 * Returns the estimate; *valid says which form was used.
 * ---------------------------------------------------------------------------------- */
double orc_shadow_triangulate(double r1, double r2, double delta, double t, double k, int* valid)
{
    if (r1 > 0.0 && r2 > 0.0 && delta > 0.0) {
        const double y = (r2 * r2 - r1 * r1 + delta * delta) / (2.0 * delta);
        const double d2 = r2 * r2 - y * y;
        if (d2 > 0.0 && t - y > 0.0) {
            if (valid) *valid = 1;
            return k * sqrt(d2) / (t - y);
        }
    }
    if (valid) *valid = 0;
    return k * r2 / t;
}

static double orc_clamp_step(const orc_shadow* s, double v)
{
    if (v < (double)s->smin) v = (double)s->smin;
    if (v > (double)s->smax) v = (double)s->smax;
    return v;
}

/* the estimate of step m from the recorded samples (plain, or triangulated when tri) */
static double orc_estimate(const orc_shadow* s, int tri, const double* tm, const double* sm, int m, int* valid)
{
    if (valid) *valid = 0;
    if (!tri || m == 0) return (double)s->k * sm[m] / tm[m];
    return orc_shadow_triangulate(sm[m - 1], sm[m], orc_clamp_step(s, sm[m - 1]), tm[m], (double)s->k, valid);
}

/* Whether X lies in the grid's box [org, org + n h] (closed), and its least distance to
 * the box faces in grid units (positive inside). */
static int orc_in_box(orc_grid g, const double X[3], double* gap)
{
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    double least = HUGE_VAL;
    int in = 1;
    for (int a = 0; a < 3; ++a) {
        const double c = (X[a] - (double)g.org[a]) / (double)g.h;
        if (c < 0.0 || c > (double)n[a]) in = 0;
        least = fmin(least, fmin(fabs(c), fabs((double)n[a] - c)));
    }
    if (gap) *gap = least;
    return in;
}

/* ------------------------------------------------------------------------------------
 * The field a march samples: one grid (L = 1), or the levels of a clip map, finest first
 * (level l's values start at f + off[l]).  A clip map is the multi-resolution field around
 * a camera that the paper proposes for large scenes: the reading used is that a point reads
 * the finest level whose box of grid-point centres holds it (grid coordinate
 * (X - org)/h - 1/2 in [0, n-1] on every axis), and the coarsest level (clamped) when none
 * does.  *gap (when given) is the least distance, in the grid units of each level tested
 * before the choice, of X from the box faces that decided it (+inf with one level).
 * ---------------------------------------------------------------------------------- */
typedef struct {
    const double* f;
    const int64_t* off;
    const orc_grid* g;
    int L;
} orc_field;

static int orc_field_level(const orc_field* F, const double X[3], double* gap)
{
    double least = HUGE_VAL;
    int l = 0;
    for (; l < F->L - 1; ++l) {
        const orc_grid* g = &F->g[l];
        const int32_t n[3] = {g->nx, g->ny, g->nz};
        int in = 1;
        for (int a = 0; a < 3; ++a) {
            const double c = (X[a] - (double)g->org[a]) / (double)g->h - 0.5;
            if (c < 0.0 || c > (double)(n[a] - 1)) in = 0;
            least = fmin(least, fmin(fabs(c), fabs((double)(n[a] - 1) - c)));
        }
        if (in) break;
    }
    if (gap) *gap = least;
    return l;
}

static double orc_field_sample(const orc_field* F, const double X[3], double grad[3])
{
    const int l = orc_field_level(F, X, NULL);
    return orc_trilinear(F->f + F->off[l], F->g[l], X, grad);
}

static void orc_field_scatter(double* gf, const orc_field* F, const double X[3], double w)
{
    const int l = orc_field_level(F, X, NULL);
    orc_trilinear_scatter(gf + F->off[l], F->g[l], X, w);
}

/* values of a clip map (or one grid) at n points X[3 n]; level[q] = the level read */
void orc_clipmap_sample(const double* f, const int64_t* off, const orc_grid* g, int32_t L, const double* X, int64_t n,
                        double* val, int32_t* level)
{
    const orc_field F = {f, off, g, L};
    for (int64_t q = 0; q < n; ++q) {
        if (level) level[q] = orc_field_level(&F, X + 3 * q, NULL);
        val[q] = orc_field_sample(&F, X + 3 * q, NULL);
    }
}

/* one pixel's march towards the unit direction l from t = t_start; records t_m and s_m
 * (arrays of s->steps, always given).  bounded: the march ends before the first sample
 * that lies outside the grid's box (section 2.4: stop beyond the scene bounds); *taken =
 * the number of samples taken.  Returns the clamped image value; *istar = index of the
 * first step attaining the minimum, or -1 when the value is the initial 1 or is clamped at
 * 0 (no gradient). */
static double orc_march_ex(const orc_field* F, const orc_shadow* s, const double l[3], double t_start, int tri,
                           int bounded, const double P[3], double* tm, double* sm, int* istar, int* taken)
{
    double t = t_start, res = 1.0;
    int best = -1, m = 0;
    for (; m < s->steps; ++m) {
        double X[3];
        for (int a = 0; a < 3; ++a) X[a] = P[a] + t * l[a];
        if (bounded && !orc_in_box(F->g[F->L - 1], X, NULL)) break;
        const double v = orc_field_sample(F, X, NULL);
        tm[m] = t;
        sm[m] = v;
        const double r = orc_estimate(s, tri, tm, sm, m, NULL);
        if (r < res) {
            res = r;
            best = m;
        }
        t += orc_clamp_step(s, v);
    }
    if (taken) *taken = m;
    if (res <= 0.0) {
        *istar = -1;
        return 0.0;
    }
    *istar = best;
    return res;
}

static double orc_march(const double* f, orc_grid g, const orc_shadow* s, const double P[3], double* tm,
                        double* sm, int* istar)
{
    const double l[3] = {(double)s->light[0], (double)s->light[1], (double)s->light[2]};
    const int64_t zero = 0;
    const orc_field F = {f, &zero, &g, 1};
    return orc_march_ex(&F, s, l, (double)s->t0, 0, 0, P, tm, sm, istar, NULL);
}

void orc_shadow_forward(const double* fine, orc_grid g, const orc_shadow* s, double* img)
{
#pragma omp parallel
    {
        double* tm = (double*)malloc(sizeof(double) * (size_t)s->steps);
        double* sm = (double*)malloc(sizeof(double) * (size_t)s->steps);
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < (int64_t)s->width * s->height; ++p) {
            double P[3];
            int istar;
            orc_pixel_origin(s, (int32_t)(p % s->width), (int32_t)(p / s->width), P);
            img[p] = orc_march(fine, g, s, P, tm, sm, &istar);
        }
        free(tm);
        free(sm);
    }
}

/* grad_fine += (d img / d fine)^T grad_img, by reverse-mode differentiation of the march */
void orc_shadow_backward(const double* fine, orc_grid g, const orc_shadow* s, const double* grad_img,
                         double* grad_fine)
{
    double* tm = (double*)malloc(sizeof(double) * (size_t)s->steps);
    double* sm = (double*)malloc(sizeof(double) * (size_t)s->steps);
    for (int64_t p = 0; p < (int64_t)s->width * s->height; ++p) {
        if (grad_img[p] == 0.0) continue;
        double P[3];
        int istar;
        orc_pixel_origin(s, (int32_t)(p % s->width), (int32_t)(p / s->width), P);
        orc_march(fine, g, s, P, tm, sm, &istar);
        if (istar < 0) continue;
        const double kk = (double)s->k;
        double sbar = grad_img[p] * kk / tm[istar];
        double tbar = -grad_img[p] * kk * sm[istar] / (tm[istar] * tm[istar]);
        for (int m = istar; m >= 0; --m) {
            double X[3], gr[3];
            for (int a = 0; a < 3; ++a) X[a] = P[a] + tm[m] * (double)s->light[a];
            orc_trilinear(fine, g, X, gr);
            orc_trilinear_scatter(grad_fine, g, X, sbar);
            tbar += sbar * ((gr[0] * (double)s->light[0] + gr[1] * (double)s->light[1]) + gr[2] * (double)s->light[2]);
            if (m == 0) break;
            /* t_m = t_{m-1} + clamp(s_{m-1}, smin, smax) */
            const double prev = sm[m - 1];
            sbar = (prev > (double)s->smin && prev < (double)s->smax) ? tbar : 0.0;
        }
    }
    free(tm);
    free(sm);
}

/* Each pixel's discrete march path, for checks that hold it fixed (finite differences of the
 * adjoint, whose derivative exists only where the path does not change): a 64-bit FNV-1a
 * hash of the minimising step (-1 when the pixel is clamped at 0 or keeps its initial 1),
 * of which earlier samples were clamped to [smin, smax], and of the trilinear cell (and the
 * in-range flags per axis) of every sample up to the minimising one.  Two fields whose paths
 * hash alike take the same branches, so the image is one smooth function between them. */
static uint64_t orc_fnv(uint64_t h, int64_t v)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (uint64_t)((v >> (8 * b)) & 0xFF);
        h *= 0x100000001B3ull;
    }
    return h;
}

void orc_shadow_path(const double* fine, orc_grid g, const orc_shadow* s, uint64_t* sig)
{
#pragma omp parallel
    {
        double* tm = (double*)malloc(sizeof(double) * (size_t)s->steps);
        double* sm = (double*)malloc(sizeof(double) * (size_t)s->steps);
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < (int64_t)s->width * s->height; ++p) {
            double P[3];
            int istar;
            orc_pixel_origin(s, (int32_t)(p % s->width), (int32_t)(p / s->width), P);
            orc_march(fine, g, s, P, tm, sm, &istar);
            uint64_t h = orc_fnv(0xCBF29CE484222325ull, istar);
            for (int m = 0; m <= istar; ++m) {
                if (m < istar) h = orc_fnv(h, sm[m] <= (double)s->smin ? 1 : (sm[m] >= (double)s->smax ? 2 : 0));
                const int32_t n[3] = {g.nx, g.ny, g.nz};
                for (int a = 0; a < 3; ++a) {
                    const double X = P[a] + tm[m] * (double)s->light[a];
                    double c = (X - (double)g.org[a]) / (double)g.h - 0.5;
                    const int inside = c > 0.0 && c < (double)(n[a] - 1);
                    if (c < 0.0) c = 0.0;
                    if (c > (double)(n[a] - 1)) c = (double)(n[a] - 1);
                    int64_t b = (int64_t)floor(c);
                    if (b > n[a] - 2) b = n[a] - 2;
                    if (b < 0) b = 0;
                    h = orc_fnv(h, 2 * b + inside);
                }
            }
            sig[p] = h;
        }
        free(tm);
        free(sm);
    }
}

/* Decision margins of each pixel's march, for comparing implementations that round
 * differently: r_margin = the least |k s_m / t_m - res| over the steps other than the
 * minimising one, together with the distances of res from the 0 clamp and from the initial
 * value 1; s_margin = the least distance of a sample s_m (m before the minimising step)
 * from the clamp bounds smin and smax; c_margin = the least distance, in grid units, of a
 * sample position (m up to the minimising step) from a cell face of the trilinear lattice
 * (the interpolant's gradient jumps there).  A pixel whose margins exceed the rounding
 * error of another implementation takes the same discrete path there. */
void orc_shadow_margin(const double* fine, orc_grid g, const orc_shadow* s, double* r_margin, double* s_margin,
                       double* c_margin)
{
#pragma omp parallel
    {
        double* tm = (double*)malloc(sizeof(double) * (size_t)s->steps);
        double* sm = (double*)malloc(sizeof(double) * (size_t)s->steps);
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < (int64_t)s->width * s->height; ++p) {
            double P[3];
            int istar;
            orc_pixel_origin(s, (int32_t)(p % s->width), (int32_t)(p / s->width), P);
            const double img = orc_march(fine, g, s, P, tm, sm, &istar);
            /* rmin = least ratio over all steps (not capped by the initial 1) */
            double rmin = HUGE_VAL, rm = HUGE_VAL, sgap = HUGE_VAL;
            int mmin = 0;
            for (int m = 0; m < s->steps; ++m) {
                const double r = (double)s->k * sm[m] / tm[m];
                if (r < rmin) {
                    rmin = r;
                    mmin = m;
                }
            }
            for (int m = 0; m < s->steps; ++m) {
                const double r = (double)s->k * sm[m] / tm[m];
                if (m != mmin) rm = fmin(rm, fabs(r - rmin));
            }
            rm = fmin(rm, fabs(rmin));
            rm = fmin(rm, fabs(1.0 - rmin));
            const int last = istar < 0 ? s->steps : istar;
            for (int m = 0; m < last; ++m)
                sgap = fmin(sgap, fmin(fabs(sm[m] - (double)s->smin), fabs(sm[m] - (double)s->smax)));
            double cgap = HUGE_VAL;
            for (int m = 0; m <= last && m < s->steps; ++m)
                for (int a = 0; a < 3; ++a) {
                    const double c = (P[a] + tm[m] * (double)s->light[a] - (double)g.org[a]) / (double)g.h - 0.5;
                    cgap = fmin(cgap, fabs(c - nearbyint(c)));
                }
            (void)img;
            r_margin[p] = rm;
            s_margin[p] = sgap;
            c_margin[p] = cgap;
        }
        free(tm);
        free(sm);
    }
}

/* ------------------------------------------------------------------------------------
 * The shadow pass with several lights, a jittered start and optional triangulation
 * (sections 2.5.2 and 3.2: three lights; a 0.05 step cap with about 128 samples; the start
 * offset jittered along the light to break up the fixed-step pattern).  Image l (of
 * nlights, each height x width, img[(l * height + b) * width + a]) marches towards
 * lights[l] from t = t0 + jitter * u, with u = (w0 >> 8) 2^-24 and w0 the first word of
 * Philox4x32-10 with counter (b * width + a, frame, l, 0xFFFFFFFF) and key (key_lo,
 * key_hi): one draw per pixel, light and frame.  The start offset is computed in binary32
 * (t0 + jitter * u, no contraction), the march in binary64.
 * ---------------------------------------------------------------------------------- */
#define ORC_MAX_LIGHTS 8
typedef struct {
    orc_shadow base;                   /* base.light is not used */
    int32_t nlights;
    float lights[ORC_MAX_LIGHTS][3];
    int32_t triangulate;
    int32_t bounded;                   /* end the march where it leaves the grid's box */
    float jitter;
    uint32_t frame;
    uint64_t key;
} orc_shadow_ex;

static double orc_shadow_start(const orc_shadow_ex* s, int64_t pixel, int32_t l)
{
    if (s->jitter == 0.0f) return (double)s->base.t0;
    const uint32_t ctr[4] = {(uint32_t)pixel, s->frame, (uint32_t)l, 0xFFFFFFFFu};
    const uint32_t key[2] = {(uint32_t)s->key, (uint32_t)(s->key >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const float u = (float)(w[0] >> 8) * (1.0f / 16777216.0f);
    volatile float ju = s->jitter * u; /* binary32 product, then a binary32 sum */
    return (double)(float)(s->base.t0 + ju);
}

static void orc_shadow_forward_field(const orc_field* F, const orc_shadow_ex* s, double* img)
{
    const orc_shadow* b = &s->base;
    const int64_t npix = (int64_t)b->width * b->height;
#pragma omp parallel
    {
        double* tm = (double*)malloc(sizeof(double) * (size_t)b->steps);
        double* sm = (double*)malloc(sizeof(double) * (size_t)b->steps);
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < npix * s->nlights; ++q) {
            const int32_t l = (int32_t)(q / npix);
            const int64_t p = q % npix;
            const double L[3] = {(double)s->lights[l][0], (double)s->lights[l][1], (double)s->lights[l][2]};
            double P[3];
            int istar, taken;
            orc_pixel_origin(b, (int32_t)(p % b->width), (int32_t)(p / b->width), P);
            img[q] = orc_march_ex(F, b, L, orc_shadow_start(s, p, l), s->triangulate, s->bounded, P, tm, sm, &istar,
                                  &taken);
        }
        free(tm);
        free(sm);
    }
}

/* grad_fine += (d img / d fine)^T grad_img.  Reverse mode of the march: at the minimising
 * step m* the estimate E depends on s_{m*} and t_{m*} (and, triangulated, on s_{m*-1}
 * directly and through delta = clamp(s_{m*-1})); then for m = m* ... 0 each s_m's adjoint is
 * scattered to its 8 grid points, t_m's adjoint gains s_m's adjoint times grad s . l, and
 * t_m = t_{m-1} + clamp(s_{m-1}) hands t_m's adjoint to s_{m-1} strictly inside
 * [smin, smax] (and to t_{m-1} always). */
static void orc_shadow_backward_field(const orc_field* F, const orc_shadow_ex* s, const double* grad_img,
                                      double* grad_fine)
{
    const orc_shadow* b = &s->base;
    const int64_t npix = (int64_t)b->width * b->height;
    double* tm = (double*)malloc(sizeof(double) * (size_t)b->steps);
    double* sm = (double*)malloc(sizeof(double) * (size_t)b->steps);
    const double smin = (double)b->smin, smax = (double)b->smax, kk = (double)b->k;
    for (int64_t q = 0; q < npix * s->nlights; ++q) {
        if (grad_img[q] == 0.0) continue;
        const int32_t l = (int32_t)(q / npix);
        const int64_t p = q % npix;
        const double L[3] = {(double)s->lights[l][0], (double)s->lights[l][1], (double)s->lights[l][2]};
        double P[3];
        int istar, taken;
        orc_pixel_origin(b, (int32_t)(p % b->width), (int32_t)(p / b->width), P);
        orc_march_ex(F, b, L, orc_shadow_start(s, p, l), s->triangulate, s->bounded, P, tm, sm, &istar, &taken);
        if (istar < 0) continue;
        const double gi = grad_img[q];
        double sbar, tbar, extra = 0.0; /* extra: direct adjoint of s_{m*-1} */
        int valid = 0;
        const double E = orc_estimate(b, s->triangulate, tm, sm, istar, &valid);
        if (valid) {
            const double r1 = sm[istar - 1], r2 = sm[istar], T = tm[istar];
            const double delta = orc_clamp_step(b, r1);
            const double y = (r2 * r2 - r1 * r1 + delta * delta) / (2.0 * delta);
            const double D = sqrt(r2 * r2 - y * y);
            const double dy_r2 = r2 / delta, dy_r1 = -r1 / delta, dy_dl = 1.0 - y / delta;
            const double dD_r2 = (r2 - y * dy_r2) / D, dD_r1 = -y * dy_r1 / D, dD_dl = -y * dy_dl / D;
            const double a = kk / (T - y), c = E / (T - y);
            sbar = gi * (a * dD_r2 + c * dy_r2);
            tbar = -gi * c;
            extra = gi * (a * dD_r1 + c * dy_r1);
            if (r1 > smin && r1 < smax) extra += gi * (a * dD_dl + c * dy_dl);
        } else {
            sbar = gi * kk / tm[istar];
            tbar = -gi * kk * sm[istar] / (tm[istar] * tm[istar]);
        }
        for (int m = istar; m >= 0; --m) {
            double X[3], gr[3];
            for (int a = 0; a < 3; ++a) X[a] = P[a] + tm[m] * L[a];
            orc_field_sample(F, X, gr);
            orc_field_scatter(grad_fine, F, X, sbar);
            tbar += sbar * ((gr[0] * L[0] + gr[1] * L[1]) + gr[2] * L[2]);
            if (m == 0) break;
            const double prev = sm[m - 1];
            sbar = (prev > smin && prev < smax) ? tbar : 0.0;
            if (m == istar) sbar += extra;
        }
    }
    free(tm);
    free(sm);
}

/* Decision margins of the pass (as orc_shadow_margin, per pixel and light), plus
 * v_margin: the least distance of the triangulation's validity tests from flipping at any
 * step (r1 and r2 from 0 in grid units of the coarsest level, d^2 relative to r2^2, t - y
 * relative to t), for a bounded march of each sample taken and the first sample outside
 * from the box faces, and with several levels of each sample from the level boxes that
 * chose its level (grid units); +inf when none applies.  A flipped validity test, exit or
 * level choice changes the image discontinuously, so v_margin matters for the image
 * itself; the other margins only for the adjoint. */
static void orc_shadow_margin_field(const orc_field* F, const orc_shadow_ex* s, double* r_margin, double* s_margin,
                                    double* c_margin, double* v_margin)
{
    const orc_shadow* b = &s->base;
    const int64_t npix = (int64_t)b->width * b->height;
#pragma omp parallel
    {
        double* tm = (double*)malloc(sizeof(double) * (size_t)b->steps);
        double* sm = (double*)malloc(sizeof(double) * (size_t)b->steps);
        double* em = (double*)malloc(sizeof(double) * (size_t)b->steps);
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < npix * s->nlights; ++q) {
            const int32_t l = (int32_t)(q / npix);
            const int64_t p = q % npix;
            const double L[3] = {(double)s->lights[l][0], (double)s->lights[l][1], (double)s->lights[l][2]};
            double P[3];
            int istar, taken;
            orc_pixel_origin(b, (int32_t)(p % b->width), (int32_t)(p / b->width), P);
            const double t_start = orc_shadow_start(s, p, l);
            orc_march_ex(F, b, L, t_start, s->triangulate, s->bounded, P, tm, sm, &istar, &taken);
            double rmin = HUGE_VAL, rm = HUGE_VAL, sgap = HUGE_VAL, cgap = HUGE_VAL, vm = HUGE_VAL;
            int mmin = 0;
            for (int m = 0; m < taken; ++m) {
                em[m] = orc_estimate(b, s->triangulate, tm, sm, m, NULL);
                if (em[m] < rmin) {
                    rmin = em[m];
                    mmin = m;
                }
            }
            for (int m = 0; m < taken; ++m)
                if (m != mmin) rm = fmin(rm, fabs(em[m] - rmin));
            rm = fmin(rm, fabs(rmin));
            rm = fmin(rm, fabs(1.0 - rmin));
            const int last = istar < 0 ? taken : istar;
            if (s->triangulate)
                for (int m = 1; m < taken; ++m) {
                    const double r1 = sm[m - 1], r2 = sm[m], delta = orc_clamp_step(b, r1);
                    vm = fmin(vm, fmin(fabs(r1), fabs(r2)) / (double)F->g[F->L - 1].h);
                    const double y = (r2 * r2 - r1 * r1 + delta * delta) / (2.0 * delta);
                    if (r2 != 0.0) vm = fmin(vm, fabs(r2 * r2 - y * y) / (r2 * r2));
                    vm = fmin(vm, fabs(tm[m] - y) / tm[m]);
                }
            if (s->bounded) {
                /* every sample position taken, and the first one outside (if any), from the box faces */
                double t = t_start;
                for (int m = 0; m <= taken && m < b->steps; ++m) {
                    if (m < taken) t = tm[m];
                    else if (m > 0) t = tm[m - 1] + orc_clamp_step(b, sm[m - 1]);
                    double X[3], gap;
                    for (int a = 0; a < 3; ++a) X[a] = P[a] + t * L[a];
                    orc_in_box(F->g[F->L - 1], X, &gap);
                    vm = fmin(vm, gap);
                }
            }
            for (int m = 0; m < last; ++m)
                sgap = fmin(sgap, fmin(fabs(sm[m] - (double)b->smin), fabs(sm[m] - (double)b->smax)));
            for (int m = 0; m < taken; ++m) {
                double X[3], lgap;
                for (int a = 0; a < 3; ++a) X[a] = P[a] + tm[m] * L[a];
                const orc_grid gl = F->g[orc_field_level(F, X, &lgap)];
                vm = fmin(vm, lgap); /* a sample near a level boundary may switch level */
                if (m <= last)
                    for (int a = 0; a < 3; ++a) {
                        const double c = (X[a] - (double)gl.org[a]) / (double)gl.h - 0.5;
                        cgap = fmin(cgap, fabs(c - nearbyint(c)));
                    }
            }
            r_margin[q] = rm;
            s_margin[q] = sgap;
            c_margin[q] = cgap;
            v_margin[q] = vm;
        }
        free(tm);
        free(sm);
        free(em);
    }
}

void orc_shadow_forward_ex(const double* fine, orc_grid g, const orc_shadow_ex* s, double* img)
{
    const int64_t zero = 0;
    const orc_field F = {fine, &zero, &g, 1};
    orc_shadow_forward_field(&F, s, img);
}

void orc_shadow_backward_ex(const double* fine, orc_grid g, const orc_shadow_ex* s, const double* grad_img,
                            double* grad_fine)
{
    const int64_t zero = 0;
    const orc_field F = {fine, &zero, &g, 1};
    orc_shadow_backward_field(&F, s, grad_img, grad_fine);
}

void orc_shadow_margin_ex(const double* fine, orc_grid g, const orc_shadow_ex* s, double* r_margin,
                          double* s_margin, double* c_margin, double* v_margin)
{
    const int64_t zero = 0;
    const orc_field F = {fine, &zero, &g, 1};
    orc_shadow_margin_field(&F, s, r_margin, s_margin, c_margin, v_margin);
}

/* the full shadow pass over a clip map (levels finest first, level l at fine + off[l]); a
 * bounded march ends where it leaves the coarsest level's grid box */
void orc_shadow_forward_clip(const double* fine, const int64_t* off, const orc_grid* g, int32_t L,
                             const orc_shadow_ex* s, double* img)
{
    const orc_field F = {fine, off, g, L};
    orc_shadow_forward_field(&F, s, img);
}

void orc_shadow_backward_clip(const double* fine, const int64_t* off, const orc_grid* g, int32_t L,
                              const orc_shadow_ex* s, const double* grad_img, double* grad_fine)
{
    const orc_field F = {fine, off, g, L};
    orc_shadow_backward_field(&F, s, grad_img, grad_fine);
}

void orc_shadow_margin_clip(const double* fine, const int64_t* off, const orc_grid* g, int32_t L,
                            const orc_shadow_ex* s, double* r_margin, double* s_margin, double* c_margin,
                            double* v_margin)
{
    const orc_field F = {fine, off, g, L};
    orc_shadow_margin_field(&F, s, r_margin, s_margin, c_margin, v_margin);
}

/* ------------------------------------------------------------------------------------
 * Adjoint of the fine field with respect to vertex positions (running-minimum mode).
 * Only a masked grid point with at least one hit depends continuously on the vertices:
 * fine = sign * t - bias, with t the distance along the ray named by its argmin record.
 * Moving vertex k of the hit triangle by d moves the plane at the hit point by b_k d, so
 * dt/dv_k = b_k n / (n . w) (n the plane normal, b the barycentrics of the hit), holding
 * the discrete state (seeds, mask, which ray and triangle give the minimum, the sign) fixed.
 * grad_verts[3 v + a] += grad_fine[p] * sign * dt/dv; binary64.
 * ---------------------------------------------------------------------------------- */
int orc_sdf_backward(const double* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                     const int32_t* vids, int64_t n, const void* bvh, const float* verts,
                     const int32_t* tris, orc_grid g, int32_t x, uint64_t seed, uint32_t obj,
                     double* grad_verts)
{
    int bad = 0;
    for (int64_t q = 0; q < n; ++q) {
        const int64_t p = vids[q];
        const uint32_t hc = hits[q];
        if (hc == 0 || grad_fine[p] == 0.0) continue;
        const uint32_t code = (uint32_t)(argmin[q] & 0xFFFFFFFFu);
        const uint32_t frame = code / (uint32_t)x, j = code % (uint32_t)x;
        float o[3], w[3], t;
        int32_t tri;
        int fr;
        orc_voxel_centre(g, p, o);
        orc_direction(seed, (uint32_t)p, frame, j, obj, w);
        if (!orc_bvh_closest(bvh, o, w, &t, &tri, &fr)) {
            ++bad;
            continue;
        }
        const double sign = (hc >> 16) > (hc & 0xFFFFu) ? -1.0 : 1.0;
        double V[3][3], O[3], W[3];
        for (int v = 0; v < 3; ++v)
            for (int a = 0; a < 3; ++a) V[v][a] = verts[3 * (int64_t)tris[3 * tri + v] + a];
        for (int a = 0; a < 3; ++a) {
            O[a] = o[a];
            W[a] = w[a];
        }
        double e1[3], e2[3], nn[3], T[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = V[1][a] - V[0][a];
            e2[a] = V[2][a] - V[0][a];
            T[a] = O[a] - V[0][a];
        }
        nn[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nn[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nn[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double nw = nn[0] * W[0] + nn[1] * W[1] + nn[2] * W[2];
        const double th = -(nn[0] * T[0] + nn[1] * T[1] + nn[2] * T[2]) / nw;  /* exact plane hit */
        double H[3], r[3];
        for (int a = 0; a < 3; ++a) H[a] = O[a] + th * W[a];
        /* barycentrics of H: areas of the sub-triangles against n */
        double bary[3];
        const double nn2 = nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2];
        for (int v = 0; v < 3; ++v) {
            const double* A = V[(v + 1) % 3];
            const double* B = V[(v + 2) % 3];
            double ab[3], ah[3];
            for (int a = 0; a < 3; ++a) {
                ab[a] = B[a] - A[a];
                ah[a] = H[a] - A[a];
            }
            r[0] = ab[1] * ah[2] - ab[2] * ah[1];
            r[1] = ab[2] * ah[0] - ab[0] * ah[2];
            r[2] = ab[0] * ah[1] - ab[1] * ah[0];
            bary[v] = (r[0] * nn[0] + r[1] * nn[1] + r[2] * nn[2]) / nn2;
        }
        const double scale = grad_fine[p] * sign / nw;
        for (int v = 0; v < 3; ++v) {
            const int64_t vi = tris[3 * tri + v];
            for (int a = 0; a < 3; ++a) grad_verts[3 * vi + a] += scale * bary[v] * nn[a];
        }
    }
    return bad;
}
