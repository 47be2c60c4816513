/*
 * rtsdf.h -- C ABI of the RTSDF signed-distance hot path for AMD Instinct MI355X (gfx950).
 *
 * Method: Tan, Chua, Koh, Bhojan, "RTSDF: Real-time Signed Distance Fields for Soft Shadow
 * Approximation in Games" (arXiv 2210.06160).  A triangle scene is voxelized into seed
 * voxels (section 2.2), jump-flooded into a coarse unsigned field (section 2.2), and the
 * grid points within a mask width of a surface (section 2.3) are refined by ray sampling
 * (section 2.1): minimum hit distance, front/back hit counts for the sign.  Frames are
 * combined by a running minimum (section 2.1) or the decay rule of Eq. 1 (section 2.5.1),
 * and a bias thickens surfaces (section 2.5.3).
 *
 * Conventions shared by every entry point
 *  - Every array pointer is a DEVICE pointer owned by the caller unless marked HOST.  The
 *    library never allocates or frees device memory and never synchronises the host: work
 *    is enqueued on `stream` (a hipStream_t passed as void*; NULL = the null stream).
 *  - Arguments are validated on the host before anything is enqueued; a non-OK status
 *    means nothing was enqueued, except RTSDF_E_DEVICE (a launch failed; outputs are
 *    unspecified).  rtsdf_last_error() returns a thread-local message for the last error.
 *  - Grids: voxel (i, j, k) has centre org + h * (i + 1/2, j + 1/2, k + 1/2) and linear
 *    index i + nx * (j + ny * k); 1 <= nx, ny, nz <= 1024; h finite and > 0.
 *  - Seed ids pack the voxel coordinates of a seed: i | j << 10 | k << 20.  RTSDF_EMPTY
 *    marks a grid point that holds no seed.
 *  - Meshes: verts float[nv][3], tris int32[nt][3] (indices into verts), wound
 *    counter-clockwise seen from outside, so (v1 - v0) x (v2 - v0) points out.
 *  - Workspaces (`work`) are caller-owned device scratch of at least the size the
 *    matching *_work_bytes() query returns; they carry nothing between calls.
 *  - Calls that overlap in time must not share output or workspace buffers.
 */
#ifndef RTSDF_H
#define RTSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTSDF_EMPTY (-1)
#define RTSDF_MAX_DIM 1024
#define RTSDF_MAX_RAYS 65535

typedef struct rtsdf_grid {
    int32_t nx, ny, nz; /* grid points per axis */
    float org[3];       /* world position of the grid's lower corner */
    float h;            /* voxel edge length (cubic voxels) */
} rtsdf_grid;

typedef int32_t rtsdf_status;
#define RTSDF_OK 0
#define RTSDF_E_ARG (-1)    /* null / aliased pointer, non-finite or non-positive parameter */
#define RTSDF_E_RANGE (-2)  /* a size or count outside its documented range */
#define RTSDF_E_SIZE (-3)   /* a workspace or output buffer smaller than required */
#define RTSDF_E_DEVICE (-4) /* a HIP call failed; see rtsdf_last_error() */

#define RTSDF_ACCUM 0 /* running minimum over frames (section 2.1) */
#define RTSDF_DECAY 1 /* Eq. 1 decay (section 2.5.1) */

/* Thread-local description of the last non-OK status ("" if none). */
const char* rtsdf_last_error(void);
/* ABI version of this header: 2. */
int32_t rtsdf_abi_version(void);

/* ---------------------------------------------------------------------------------------
 * rtsdf_voxelize -- section 2.2 seeding, at the resolution of the distance field itself:
 * every grid point whose closed voxel cube meets a closed triangle
 * becomes a seed holding its own id; every other grid point is set to RTSDF_EMPTY.
 * Vertices are snapped to 1/256 voxel, X = rint(((v - org) / h) * 256) in binary32, and the
 * overlap is decided exactly in integers (separating axes of a box and a triangle).
 * Triangles with a snapped coordinate beyond +-2^19 (2048 voxels from org) are skipped.
 *   verts  [nv*3] float     tris [nt*3] int32 (each index in [0, nv); not checked on device)
 *   seeds  [N] int32 out    work [rtsdf_voxelize_work_bytes(nt)]
 * nt = 0 is legal (all RTSDF_EMPTY).  Errors: E_ARG (null pointers, bad grid), E_RANGE
 * (dims, nv/nt < 0), E_SIZE (work too small).
 * ------------------------------------------------------------------------------------- */
size_t rtsdf_voxelize_work_bytes(int32_t nt);
rtsdf_status rtsdf_voxelize(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                            rtsdf_grid g, int32_t* seeds, void* work, size_t work_bytes,
                            void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_jfa -- section 2.2 jump flooding.  Pass s uses offset k = steps[s]: every grid
 * point p keeps its stored seed, then queries p + k*e for the 26 offsets
 * e in {-1,0,1}^3 \ {0} in the order ez, ey, ex ascending; a query inside the grid that
 * holds a seed replaces the stored seed only if that seed is strictly closer (squared
 * voxel distance).  Each pass reads one buffer and writes the other (ping-pong), so the
 * result does not depend on scheduling.
 *   seeds    [N] int32 in: voxelize output; also ping-pong buffer
 *   scratch  [N] int32 ping-pong buffer, must not alias seeds
 *   steps    HOST int32[nsteps], each in [1, 1024]; nsteps in [0, 64]
 *   result_in_scratch  HOST int32 out: 1 if the result is in scratch (nsteps odd), else 0
 * The result holds packed ids and RTSDF_EMPTY like the input; the other buffer is left with
 * an intermediate pass's output in an internal encoding (the bitwise complement of each
 * id) and means nothing to the caller.
 * Errors: E_ARG (null / aliased pointers, bad grid, step < 1), E_RANGE (dims, nsteps).
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_jfa(int32_t* seeds, int32_t* scratch, rtsdf_grid g, const int32_t* steps,
                       int32_t nsteps, int32_t* result_in_scratch, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_band -- section 2.3 ray mask: the grid points whose stored seed is within
 * band_vox voxels (d2 <= band_vox^2, exact integers), listed in increasing linear index.
 *   seeds      [N] int32 jump-flooding result
 *   band_list  [N] int32 out: voxel linear indices; entries past the count are unspecified
 *   band_count [1] int32 out (device): number of listed voxels
 *   work       [rtsdf_band_work_bytes(g)]
 * Errors: E_ARG, E_RANGE (band_vox outside [0, 2048]), E_SIZE.
 * ------------------------------------------------------------------------------------- */
size_t rtsdf_band_work_bytes(rtsdf_grid g);
rtsdf_status rtsdf_band(const int32_t* seeds, rtsdf_grid g, int32_t band_vox, int32_t* band_list,
                        int32_t* band_count, void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_build_bvh -- acceleration structure for the ray sampling of section 2.1 (the
 * paper uses the graphics driver's hierarchy; CDNA has no ray-tracing units, so this is
 * a software hierarchy built from 30-bit Morton codes of triangle centroids and a stable
 * radix sort, then either
 *   RTSDF_BVH_LBVH: the Karras (2012) binary radix tree with a bottom-up box refit (fast
 *                   to build; for per-frame rebuilds), or
 *   RTSDF_BVH_PLOC: parallel locally-ordered clustering (Meister & Bittner 2018: merge
 *                   mutual nearest neighbours by merged-box area within +-16 clusters
 *                   in Morton order; about 30 % fewer node visits per ray),
 * collapsed to a 4-wide hierarchy whose child boxes are quantised to 8 bits per plane
 * (rounded outward).  Triangle boxes are widened by 2 * h/256 so that traversal returns
 * exactly the brute-force closest hit of the hit test described at rtsdf_raysample,
 * whichever tree is built.  The blob is self-contained (it copies the
 * triangles).
 *   bvh   [rtsdf_bvh_bytes(nt)] out      work [rtsdf_bvh_work_bytes(nt)]
 * Errors: E_ARG, E_RANGE (nt outside [0, 2^26], unknown method), E_SIZE.
 * ------------------------------------------------------------------------------------- */
#define RTSDF_BVH_LBVH 0
#define RTSDF_BVH_PLOC 1
size_t rtsdf_bvh_bytes(int32_t nt);
size_t rtsdf_bvh_work_bytes(int32_t nt);
rtsdf_status rtsdf_build_bvh(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                             rtsdf_grid g, int32_t method, void* bvh, size_t bvh_bytes, void* work,
                             size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_reset_accum -- sets dmin = +inf, hits = 0 and (if non-NULL) argmin = ~0 for n
 * entries (a kernel, not a memset, so it may be captured into a graph).
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_reset_accum(float* dmin, uint32_t* hits, uint64_t* argmin, int64_t n,
                               void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_raysample -- section 2.1 ray sampling of the masked grid points for one frame.
 * For listed voxel p and ray j < rays_per_voxel: the direction is uniform on the sphere
 * (Philox4x32-10 with key rng_key and counter (p, frame, j, obj << 8 | attempt), then
 * Marsaglia's 1972 rejection method); the ray starts at p's centre; the hit is
 * Moller-Trumbore in binary32 (t > 0, and the computed hit point inside the triangle's
 * box widened by h/256); the closest hit is the least (t, triangle index).  With no
 * maximum distance, every ray that hits votes: front face (dot(dir, normal) < 0) adds 1,
 * back face adds 1 << 16 to hits[p]; dmin[p] = min(dmin[p], t); argmin[p] =
 * min(argmin[p], bits(t) << 32 | (frame * rays_per_voxel + j)).  Results do not depend on
 * scheduling.  The caller keeps (front + back) <= 65535 across frames.
 *   band_list/band_count  rtsdf_band output; band_capacity HOST bound on the count
 *   dmin [N] float, hits [N] uint32, argmin [N] uint64 or NULL: accumulated in place
 *   obj  object index (< 2^24) mixed into the counter; 0 for a single scene
 *   work [rtsdf_raysample_work_bytes(band_capacity, rays_per_voxel)]: work cursors;
 *        nothing is carried between calls
 * The listed voxels must be distinct (rtsdf_band lists are).
 * Errors: E_ARG, E_RANGE (rays_per_voxel outside [1, 65535], obj >= 2^24), E_SIZE.
 * ------------------------------------------------------------------------------------- */
size_t rtsdf_raysample_work_bytes(int64_t band_capacity, int32_t rays_per_voxel);
rtsdf_status rtsdf_raysample(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                             const int32_t* band_count, int64_t band_capacity,
                             int32_t rays_per_voxel, uint64_t rng_key, uint32_t frame,
                             uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin,
                             void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_raysample_frame_device -- rtsdf_raysample with the frame index read from device
 * memory (`frame`, one uint32, device pointer) when the kernel runs rather than passed by
 * value, so that a per-frame chain recorded once into a HIP graph can be replayed for
 * every frame of a sequence (section 2.5.1 updates the field each frame) with only the
 * frame word changed between replays.  Results and errors as rtsdf_raysample (E_ARG also
 * for a NULL frame).
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_raysample_frame_device(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                                          const int32_t* band_count, int64_t band_capacity,
                                          int32_t rays_per_voxel, uint64_t rng_key,
                                          const uint32_t* frame, uint32_t obj, float* dmin,
                                          uint32_t* hits, uint64_t* argmin, void* work,
                                          size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_raysample_noalloc -- rtsdf_raysample without a work argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments (minus work / work_bytes), same
 * results, same errors, plus E_SIZE if the call's work cursors would exceed the static
 * scratch (4096 bytes; the cursors take 1 KiB whatever the input size) and E_DEVICE if
 * the scratch's device address cannot be looked up.
 * The cursors live in a static device array of 4096 bytes that the library holds on each
 * GPU it runs on until the process ends; its device address is looked up once per GPU on
 * the first call there.  The call allocates and frees nothing.  Every call on one GPU
 * shares that GPU's array (each call clears it first, with a kernel): calls on one GPU that
 * overlap in time -- on different streams, or from different host threads -- race and give
 * wrong results; serialise them.
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_raysample_noalloc(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                                     const int32_t* band_count, int64_t band_capacity,
                                     int32_t rays_per_voxel, uint64_t rng_key, uint32_t frame,
                                     uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin,
                                     void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_combine -- the fine field, elementwise over all N grid points.
 *   u = h * sqrt(d2) (binary32; +inf without a seed), c = u - beta (section 2.2), in band
 *   iff d2 <= band_vox^2 (section 2.3), sign negative iff back hits > front hits (2.1).
 *   RTSDF_ACCUM: in band with hits, +-dmin; otherwise c.
 *   RTSDF_DECAY (Eq. 1 on magnitudes): in band m = min(alpha * m_prev + (1 - alpha) * u,
 *     r) with r = dmin or +inf without hits, sign = majority or the previous sign on a tie,
 *     state = sign * m; outside the band state = +u and the value is c.  first_frame != 0
 *     (or a non-finite state) starts from m_prev = u with a positive sign.
 *   fine = value - bias (section 2.5.3: a positive bias thickens surfaces).
 *   consume != 0: after reading, grid points with hits != 0 are reset to dmin = +inf,
 *   hits = 0, ready for the next frame.
 *   seeds [N] int32; dmin [N] float, hits [N] uint32 (written only if consume);
 *   state [N] float inout (DECAY only; may be NULL for ACCUM); fine [N] float out
 * Errors: E_ARG (alpha outside [0, 1] in DECAY, non-finite beta/bias, NULL state in
 * DECAY), E_RANGE (band_vox outside [0, 2048], mode).
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_combine(const int32_t* seeds, float* dmin, uint32_t* hits, rtsdf_grid g,
                           int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                           int32_t first_frame, int32_t consume, float* state, float* fine,
                           void* stream);

/* ---------------------------------------------------------------------------------------
 * Two-level field -- jump flooding on a coarse grid, rays and the combined field on a grid
 * refined by an integer ratio r over the same box (section 2.3 masks a traced field finer
 * than the flooded one; section 2.5.1 floods 128^3 beside a 256^3 traced field).
 * rtsdf_refine_grid (host only): fine = (r nx, r ny, r nz) points, same origin,
 *   h_fine = h / r in binary32.  Fine point (x, y, z) lies in coarse point
 *   (x / r, y / r, z / r) (integer division) and takes that point's coarse distance u,
 *   outside value c and band test.  Errors: E_ARG (NULL fine), E_RANGE (r < 1 or a fine
 *   dimension above RTSDF_MAX_DIM; the coarse grid as rtsdf_grid).
 * rtsdf_band_refined: the mask of rtsdf_band on the fine grid -- the fine points whose
 *   coarse parent is in band -- listed by fine linear index in increasing order.
 *   seeds [N_coarse] int32; band_list [N_fine] out; band_count [1] out (device);
 *   work [rtsdf_band_refined_work_bytes(coarse, r)].  Errors as rtsdf_band, plus r.
 * rtsdf_combine_refined: rtsdf_combine on the fine grid.  seeds [N_coarse]; dmin, hits,
 *   state and fine are [N_fine] (the fine grid's ray-sampling accumulators); u is computed
 *   with the coarse h.  Errors as rtsdf_combine, plus r.
 * Ray sampling and the vertex adjoint run unchanged on the fine grid and its mask
 * (rtsdf_raysample / rtsdf_backward with g = the refined grid); ratio 1 is the
 * single-level chain.
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_refine_grid(rtsdf_grid coarse, int32_t ratio, rtsdf_grid* fine);
size_t rtsdf_band_refined_work_bytes(rtsdf_grid coarse, int32_t ratio);
rtsdf_status rtsdf_band_refined(const int32_t* seeds, rtsdf_grid coarse, int32_t ratio, int32_t band_vox,
                                int32_t* band_list, int32_t* band_count, void* work, size_t work_bytes,
                                void* stream);
rtsdf_status rtsdf_combine_refined(const int32_t* seeds, float* dmin, uint32_t* hits, rtsdf_grid coarse,
                                   int32_t ratio, int32_t band_vox, float beta, float bias, int32_t mode,
                                   float alpha, int32_t first_frame, int32_t consume, float* state,
                                   float* fine, void* stream);

/* ---------------------------------------------------------------------------------------
 * Soft shadows by sphere tracing the fine field (section 2.4; step bounds of section
 * 2.5.2, start offset of section 2.5.3).  The receiver is the plane y = `y`; pixel (a, b)
 * (a < width along x, b < height along z; img[b * width + a]) starts at
 * P = (x0 + (a + 1/2) dx, y, z0 + (b + 1/2) dz) and marches towards the light along the
 * unit vector `light`: t = t0, res = 1; each of `steps` steps samples s = fine at P + t l
 * (trilinear over the grid points, the sample position clamped to the grid's box of
 * centres), sets res = min(res, k s / t) and advances t by s clamped to [smin, smax].
 * The pixel is clamp(res, 0, 1).  Binary32 arithmetic.
 * ------------------------------------------------------------------------------------- */
#define RTSDF_MAX_SHADOW_STEPS 256
#define RTSDF_MAX_IMAGE 16384

typedef struct rtsdf_shadow {
    int32_t width, height;  /* pixels, each in [0, 16384] */
    float x0, z0, dx, dz;   /* pixel lattice on the receiver plane */
    float y;                /* receiver plane height */
    float light[3];         /* unit direction towards the light */
    float k;                /* penumbra sharpness, > 0 */
    int32_t steps;          /* march steps, [1, 256] */
    float smin, smax;       /* step clamp, 0 < smin <= smax */
    float t0;               /* start offset along the light direction, > 0 */
} rtsdf_shadow;

/* rtsdf_shadow_forward -- the shadow image of the fine field.
 *   fine [N] float (rtsdf_combine output)     img [height * width] float out (may be NULL
 *   when the image has no pixels)
 * Errors: E_ARG (null pointers, bad grid, non-finite or out-of-range parameters),
 * E_RANGE (image size, steps). */
rtsdf_status rtsdf_shadow_forward(const float* fine, rtsdf_grid g, rtsdf_shadow s, float* img,
                                  void* stream);

/* rtsdf_shadow_backward -- reverse-mode derivative of rtsdf_shadow_forward:
 * grad_fine += (d img / d fine)^T grad_img.  Per pixel, m* is the first step attaining the
 * minimum of k s / t; pixels whose value is the initial 1 or is clamped at 0 contribute
 * nothing.  Otherwise the adjoint of res = k s_m* / t_m* is carried back over m = m*..0
 * through t_{m+1} = t_m + clamp(s_m) (the clamp passes the derivative only strictly
 * inside [smin, smax]) and through each trilinear sample to its 8 grid points.
 *   fine [N] float (the forward's input)   grad_img [height * width] float
 *   grad_fine [N] float, ACCUMULATED with binary32 atomic adds (summation order varies)
 * Errors: as rtsdf_shadow_forward. */
rtsdf_status rtsdf_shadow_backward(const float* fine, rtsdf_grid g, rtsdf_shadow s,
                                   const float* grad_img, float* grad_fine, void* stream);

/* ---------------------------------------------------------------------------------------
 * The full shadow pass (sections 2.5.2 and 3.2): several lights in one launch, the start
 * offset jittered along the light, and optionally the two-sample triangulation of the
 * closest approach (after Aaltonen 2018).  Image l marches towards lights[l] exactly as
 * rtsdf_shadow_forward, except:
 *  - start: t = t0 + jitter * u in binary32, u = (w0 >> 8) * 2^-24 with w0 the first word
 *    of Philox4x32-10 for counter (b * width + a, frame, l, 0xFFFFFFFF) and key; jitter 0
 *    starts at t0;
 *  - triangulate != 0: from the second step on, the estimate k s / t is replaced by the
 *    closest approach both samples allow: r1 = s_{m-1}, r2 = s_m bound empty spheres one
 *    step delta = clamp(r1, smin, smax) apart; their intersection circle lies
 *    y = (r2^2 - r1^2 + delta^2) / (2 delta) behind the later sample with radius
 *    d = sqrt(r2^2 - y^2), and the estimate is k d / (t_m - y) when r1 > 0, r2 > 0,
 *    d^2 > 0 and t_m - y > 0, else k r2 / t_m.
 *  - bounded != 0: the march ends before the first sample point outside the grid's box
 *    [org, org + n h] (per axis, closed), so that a long march does not keep sampling the
 *    clamped border of the field (section 2.4 stops beyond the scene bounds).
 * The adjoint is the reverse march of rtsdf_shadow_backward; triangulated, the minimising
 * estimate also depends on s_{m*-1} directly and through delta.
 *   base: receiver lattice, k, steps, step bounds and t0 as rtsdf_shadow (base.light is
 *         ignored but must be finite); lights: nlights unit directions, 1 <= nlights <= 8;
 *   jitter >= 0 (world units); img / grad_img [nlights][height][width] float.
 * s is a HOST pointer.  Errors: as rtsdf_shadow_forward, plus E_RANGE (nlights) and E_ARG
 * (non-finite light or jitter < 0).
 * ------------------------------------------------------------------------------------- */
#define RTSDF_MAX_LIGHTS 8

typedef struct rtsdf_shadow_ex {
    rtsdf_shadow base;
    int32_t nlights;
    float lights[RTSDF_MAX_LIGHTS][3];
    int32_t triangulate;
    int32_t bounded;
    float jitter;
    uint32_t frame;
    uint64_t key;
} rtsdf_shadow_ex;

rtsdf_status rtsdf_shadow_forward_ex(const float* fine, rtsdf_grid g, const rtsdf_shadow_ex* s, float* img,
                                     void* stream);
rtsdf_status rtsdf_shadow_backward_ex(const float* fine, rtsdf_grid g, const rtsdf_shadow_ex* s,
                                      const float* grad_img, float* grad_fine, void* stream);

/* ---------------------------------------------------------------------------------------
 * rtsdf_backward -- derivative of the running-minimum fine field (RTSDF_ACCUM, section
 * 2.1) with respect to vertex positions, the discrete state held fixed (seeds, mask, the
 * argmin ray of each grid point, its closest triangle and the sign).  A masked grid point
 * with hits has fine = sign * t - bias, t the distance along the ray its argmin record
 * names; that ray is traced again (same direction and hit rule as rtsdf_raysample) to its
 * closest triangle, and vertex k of that triangle receives
 *   grad_fine[p] * sign * b_k * n / (n . w)
 * (n = (v1 - v0) x (v2 - v0), w the ray direction, b the barycentrics of the hit).  Grid
 * points outside the mask or without hits contribute nothing (the coarse field is
 * piecewise constant in the vertices).
 *   grad_fine [N] float; hits [N], argmin [N]: the accumulators after the last frame
 *   band_list/band_count/band_capacity: the rtsdf_band output used by the forward
 *   bvh: rtsdf_build_bvh output for these tris; tris [nt*3] int32 (indices < nv)
 *   rays_per_voxel, rng_key, obj: as passed to rtsdf_raysample
 *   grad_verts [nv*3] float, ACCUMULATED with binary32 atomic adds
 * Errors: E_ARG, E_RANGE (rays_per_voxel, obj, nv < 0, nt outside [0, 2^26]).
 * ------------------------------------------------------------------------------------- */
rtsdf_status rtsdf_backward(const float* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                            const int32_t* band_list, const int32_t* band_count,
                            int64_t band_capacity, const void* bvh, const int32_t* tris,
                            int32_t nv, int32_t nt, rtsdf_grid g, int32_t rays_per_voxel,
                            uint64_t rng_key, uint32_t obj, float* grad_verts, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched objects -- many independent scenes, each with its own mesh and grid, run by one
 * launch per stage (per JFA pass) instead of one call chain per object; the dispatch cost
 * the paper attributes to its per-pass calls (section 3.1.2) is paid once per batch.  Each
 * object computes exactly what the single-object calls compute for it (with obj = its
 * index in the batch), so seeds, masks, hit counts and argmin records are bit-identical.
 *
 * Layout of the concatenated arrays (all in object order):
 *   verts [sum nv][3], tris [sum nt][3] with indices local to the object's vertices;
 *   per-grid-point arrays (seeds, dmin, hits, argmin, fine, grad_fine): object o's grid
 *   starts at voxel offset V_o = sum over p < o of roundup(N_p, RTSDF_BATCH_ALIGN); the
 *   voxels between objects are padding that no call reads or writes;
 *   mask lists hold indices into these concatenated arrays;
 *   hierarchies: object o's blob starts at byte offset B_o = sum over p < o of
 *   roundup(rtsdf_bvh_bytes(nt_p), 256).
 * A plan (rtsdf_batch_plan) records the layout and the launch tables.  It is caller-owned
 * memory in two copies of rtsdf_batch_plan_bytes(nobj) bytes, one in host memory (read
 * by every batched call to size its launches) and one in device memory (read by the
 * kernels); the host copy remembers the device copy's address.  Both must stay unchanged
 * while calls that use them are in flight.
 * ------------------------------------------------------------------------------------- */
#define RTSDF_BATCH_ALIGN 4096
#define RTSDF_MAX_OBJECTS 65536

typedef struct rtsdf_object {
    rtsdf_grid g;          /* the object's grid */
    int32_t nv, nt;        /* its vertices and triangles */
    int32_t band_vox;      /* mask width in voxels, [0, 2048] */
    int32_t extra_passes;  /* trailing JFA passes with offset 1 after 2^(ceil(log2 max dim)-1)..1, [0, 8] */
    float beta, bias;      /* combine parameters, world units of this object */
} rtsdf_object;

typedef struct rtsdf_batch_sizes {
    int64_t voxels;        /* length of the concatenated per-grid-point arrays */
    int64_t verts, tris;   /* rows of the concatenated verts and tris */
    size_t bvh_bytes;      /* bytes of the concatenated hierarchies */
    size_t work_bytes;     /* workspace every batched call accepts */
    int32_t max_passes;    /* JFA passes of the longest object */
} rtsdf_batch_sizes;

size_t rtsdf_batch_plan_bytes(int32_t nobj);
/* Builds the plan from objs (HOST, nobj in [1, 65536]) into plan_host (host work only) and
 * records plan_device as the address of its device copy.  Errors: E_ARG (null pointers, a
 * bad grid or parameter), E_RANGE (counts; the batch must stay below 2^31 grid points and
 * vertices and 2^26 triangles), E_SIZE (plan_bytes too small). */
rtsdf_status rtsdf_batch_plan(const rtsdf_object* objs, int32_t nobj, void* plan_host, void* plan_device,
                              size_t plan_bytes, rtsdf_batch_sizes* sizes);
/* Copies the host plan to its device copy on `stream` and waits for the copy (this call
 * synchronizes the stream).  Errors: E_ARG (not a plan), E_DEVICE. */
rtsdf_status rtsdf_batch_upload(const void* plan_host, void* stream);
/* Layout query: object o's voxel offset V_o and hierarchy byte offset B_o (HOST outs). */
rtsdf_status rtsdf_batch_offsets(const void* plan_host, int32_t o, int64_t* vox_offset, size_t* bvh_offset);

/* As rtsdf_voxelize per object.  An object with an odd number of JFA passes receives its
 * seeds in `scratch`, the others in `seeds`, so that rtsdf_jfa_batched leaves every
 * result in `seeds`.  seeds, scratch [sizes.voxels] int32; work [sizes.work_bytes]. */
rtsdf_status rtsdf_voxelize_batched(const void* plan_host, const float* verts, const int32_t* tris,
                                    int32_t* seeds, int32_t* scratch, void* work, size_t work_bytes,
                                    void* stream);
/* As rtsdf_jfa per object with its own offsets; one launch per pass over every object
 * still flooding; the results end in `seeds` (see rtsdf_voxelize_batched), and `scratch`
 * is left with intermediate passes in an internal encoding (as for rtsdf_jfa). */
rtsdf_status rtsdf_jfa_batched(const void* plan_host, int32_t* seeds, int32_t* scratch, void* stream);
/* As rtsdf_band per object with its own mask width; one list over the concatenated grid
 * points, increasing.  band_list [sizes.voxels] int32, band_count [1] int32 (device). */
rtsdf_status rtsdf_band_batched(const void* plan_host, const int32_t* seeds, int32_t* band_list,
                                int32_t* band_count, void* work, size_t work_bytes, void* stream);
/* As rtsdf_build_bvh per object (the object's grid sets the hit padding); every phase of
 * the build is one launch for all objects (a segmented sort, then the tree of each object
 * in its own segment). */
rtsdf_status rtsdf_build_bvh_batched(const void* plan_host, const float* verts, const int32_t* tris,
                                     int32_t method, void* bvh, size_t bvh_bytes, void* work, size_t work_bytes,
                                     void* stream);
/* As rtsdf_raysample per object with obj = the object's index; one launch for the batch. */
rtsdf_status rtsdf_raysample_batched(const void* plan_host, const void* bvh, const int32_t* band_list,
                                     const int32_t* band_count, int64_t band_capacity, int32_t rays_per_voxel,
                                     uint64_t rng_key, uint32_t frame, float* dmin, uint32_t* hits,
                                     uint64_t* argmin, void* work, size_t work_bytes, void* stream);
/* As rtsdf_combine in RTSDF_ACCUM mode per object (its band_vox, beta, bias). */
rtsdf_status rtsdf_combine_batched(const void* plan_host, const int32_t* seeds, const float* dmin,
                                   const uint32_t* hits, float* fine, void* stream);
/* As rtsdf_backward per object; grad_verts [sizes.verts * 3] accumulated. */
rtsdf_status rtsdf_backward_batched(const void* plan_host, const float* grad_fine, const uint32_t* hits,
                                    const uint64_t* argmin, const int32_t* band_list, const int32_t* band_count,
                                    int64_t band_capacity, const void* bvh, const int32_t* tris,
                                    int32_t rays_per_voxel, uint64_t rng_key, float* grad_verts, void* stream);

/* ---------------------------------------------------------------------------------------
 * Clip map -- several resolutions of the field around a camera, for scenes larger than one
 * grid can cover (the paper's future-work section proposes it without a design).  Level l
 * is a grid of n^3 points of size h0 * 2^l; a clip map is a batch plan whose objects are its
 * levels, finest first (built and run with the *_batched calls, every level holding the same
 * mesh), and these calls read the concatenated fine field of such a batch.
 * rtsdf_clipmap_levels (host only): the level grids around `camera`: level l's origin on
 *   each axis is (floor(c / h) - n/2) * h in binary32 with h = h0 * 2^l, so a level stays
 *   fixed while the camera moves inside one of its voxels and lies inside the next level's
 *   box.  camera HOST float[3], grids HOST out [levels].  Errors: E_ARG (NULL, h0 not finite
 *   and > 0, camera not finite), E_RANGE (n not even in [4, RTSDF_MAX_DIM], levels outside
 *   [1, RTSDF_MAX_CLIP_LEVELS]).
 * Sampling rule: a point reads the finest level whose box of grid-point centres holds it
 *   (grid coordinate (X - org)/h - 1/2 in [0, n-1] on every axis), trilinearly as
 *   rtsdf_shadow_forward samples one grid; when no level holds it, the coarsest (clamped).
 * rtsdf_clipmap_sample: values (and, if levels != NULL, the level read) at n points
 *   (points [n][3] float, values [n] float, levels [n] int32, all device).
 * rtsdf_shadow_forward_clip / rtsdf_shadow_backward_clip: the full shadow pass
 *   (rtsdf_shadow_forward_ex) marching through the clip map by the sampling rule; a bounded
 *   march ends at the coarsest level's box; the adjoint accumulates into the concatenated
 *   grad_fine of the level each sample read.
 *   plan: HOST copy of the batch plan whose objects are the levels (1..RTSDF_MAX_CLIP_LEVELS).
 * Errors: E_ARG (NULL pointers, a bad plan, parameters as rtsdf_shadow_forward_ex), E_RANGE
 * (number of levels, n < 0).
 * ------------------------------------------------------------------------------------- */
#define RTSDF_MAX_CLIP_LEVELS 8

rtsdf_status rtsdf_clipmap_levels(const float* camera, float h0, int32_t n, int32_t levels, rtsdf_grid* grids);
rtsdf_status rtsdf_clipmap_sample(const void* plan, const float* fine, const float* points, int64_t n, float* values,
                                  int32_t* levels, void* stream);
rtsdf_status rtsdf_shadow_forward_clip(const void* plan, const float* fine, const rtsdf_shadow_ex* s, float* img,
                                       void* stream);
rtsdf_status rtsdf_shadow_backward_clip(const void* plan, const float* fine, const rtsdf_shadow_ex* s,
                                        const float* grad_img, float* grad_fine, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RTSDF_H */
