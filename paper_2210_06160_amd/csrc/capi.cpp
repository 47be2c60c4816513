// C ABI of librtsdf.so: host-side validation, then the HIP launchers.  No exception or
// allocation crosses this layer; every failure becomes an rtsdf_status plus a thread-local
// message.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "internal.h"

namespace {

thread_local char g_err[512] = "";

rtsdf_status fail(rtsdf_status code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

rtsdf_status ok()
{
    g_err[0] = '\0';
    return RTSDF_OK;
}

rtsdf_status device(hipError_t e, const char* what)
{
    if (e == hipSuccess) return ok();
    return fail(RTSDF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

rtsdf_status check_grid(const rtsdf_grid& g)
{
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > RTSDF_MAX_DIM || g.ny > RTSDF_MAX_DIM ||
        g.nz > RTSDF_MAX_DIM)
        return fail(RTSDF_E_RANGE, "grid dims %d x %d x %d outside [1, %d]", g.nx, g.ny, g.nz,
                    RTSDF_MAX_DIM);
    if (!std::isfinite(g.h) || !(g.h > 0.0f))
        return fail(RTSDF_E_ARG, "voxel size h must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g.org[a])) return fail(RTSDF_E_ARG, "grid origin must be finite");
    return RTSDF_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

rtsdf_status check_shadow(const rtsdf_shadow& s)
{
    if (s.width < 0 || s.height < 0 || s.width > RTSDF_MAX_IMAGE || s.height > RTSDF_MAX_IMAGE)
        return fail(RTSDF_E_RANGE, "image %d x %d outside [0, %d]^2", s.width, s.height, RTSDF_MAX_IMAGE);
    if (s.steps < 1 || s.steps > RTSDF_MAX_SHADOW_STEPS)
        return fail(RTSDF_E_RANGE, "steps %d outside [1, %d]", s.steps, RTSDF_MAX_SHADOW_STEPS);
    const float v[] = {s.x0, s.z0, s.dx, s.dz, s.y, s.light[0], s.light[1], s.light[2], s.k, s.smin, s.smax, s.t0};
    for (float f : v)
        if (!std::isfinite(f)) return fail(RTSDF_E_ARG, "shadow parameters must be finite");
    if (!(s.k > 0.0f) || !(s.t0 > 0.0f) || !(s.smin > 0.0f) || !(s.smax >= s.smin))
        return fail(RTSDF_E_ARG, "need k > 0, t0 > 0 and 0 < smin <= smax");
    return RTSDF_OK;
}

}  // namespace

extern "C" {

const char* rtsdf_last_error(void) { return g_err; }

int32_t rtsdf_abi_version(void) { return 1; }

size_t rtsdf_voxelize_work_bytes(int32_t nt) { return nt < 0 ? 0 : rtsdf::voxelize_work_bytes(nt); }

rtsdf_status rtsdf_voxelize(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                            rtsdf_grid g, int32_t* seeds, void* work, size_t work_bytes, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (nv < 0 || nt < 0) return fail(RTSDF_E_RANGE, "nv and nt must be >= 0");
    if (!seeds) return fail(RTSDF_E_ARG, "seeds is NULL");
    if (nt > 0 && (!verts || !tris || !work)) return fail(RTSDF_E_ARG, "verts, tris or work is NULL");
    if (nt > 0 && nv == 0) return fail(RTSDF_E_RANGE, "triangles given but no vertices");
    if (nt > 0 && work_bytes < rtsdf::voxelize_work_bytes(nt))
        return fail(RTSDF_E_SIZE, "voxelize work %zu < %zu bytes", work_bytes, rtsdf::voxelize_work_bytes(nt));
    return device(rtsdf::voxelize(verts, tris, nt, g, seeds, work, as_stream(stream)), "voxelize");
}

rtsdf_status rtsdf_jfa(int32_t* seeds, int32_t* scratch, rtsdf_grid g, const int32_t* steps,
                       int32_t nsteps, int32_t* result_in_scratch, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!seeds || !scratch || !result_in_scratch) return fail(RTSDF_E_ARG, "NULL pointer");
    if (seeds == scratch) return fail(RTSDF_E_ARG, "seeds and scratch must not alias");
    if (nsteps < 0 || nsteps > 64) return fail(RTSDF_E_RANGE, "nsteps %d outside [0, 64]", nsteps);
    if (nsteps > 0 && !steps) return fail(RTSDF_E_ARG, "steps is NULL");
    for (int32_t i = 0; i < nsteps; ++i)
        if (steps[i] < 1 || steps[i] > RTSDF_MAX_DIM)
            return fail(RTSDF_E_ARG, "steps[%d] = %d outside [1, %d]", i, steps[i], RTSDF_MAX_DIM);
    int32_t* a = seeds;
    int32_t* b = scratch;
    for (int32_t i = 0; i < nsteps; ++i) {
        hipError_t e = rtsdf::jfa_pass(a, b, g, steps[i], as_stream(stream));
        if (e != hipSuccess) return device(e, "jfa pass");
        std::swap(a, b);
    }
    *result_in_scratch = (nsteps & 1) ? 1 : 0;
    return ok();
}

size_t rtsdf_band_work_bytes(rtsdf_grid g)
{
    if (check_grid(g) != RTSDF_OK) return 0;
    return rtsdf::band_work_bytes(g);
}

rtsdf_status rtsdf_band(const int32_t* seeds, rtsdf_grid g, int32_t band_vox, int32_t* band_list,
                        int32_t* band_count, void* work, size_t work_bytes, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!seeds || !band_list || !band_count || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (band_vox < 0 || band_vox > 2048) return fail(RTSDF_E_RANGE, "band_vox %d outside [0, 2048]", band_vox);
    if (work_bytes < rtsdf::band_work_bytes(g))
        return fail(RTSDF_E_SIZE, "band work %zu < %zu bytes", work_bytes, rtsdf::band_work_bytes(g));
    return device(rtsdf::band(seeds, g, band_vox, band_list, band_count, work, as_stream(stream)), "band");
}

size_t rtsdf_bvh_bytes(int32_t nt) { return nt < 0 ? 0 : rtsdf::bvh_bytes(nt); }
size_t rtsdf_bvh_work_bytes(int32_t nt) { return nt < 0 ? 0 : rtsdf::bvh_work_bytes(nt); }

rtsdf_status rtsdf_build_bvh(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                             rtsdf_grid g, void* bvh, size_t bvh_bytes, void* work, size_t work_bytes,
                             void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (nv < 0 || nt < 0 || nt > (1 << 26)) return fail(RTSDF_E_RANGE, "nt %d outside [0, 2^26]", nt);
    if (!bvh) return fail(RTSDF_E_ARG, "bvh is NULL");
    if (nt > 0 && (!verts || !tris || !work)) return fail(RTSDF_E_ARG, "verts, tris or work is NULL");
    if (nt > 0 && nv == 0) return fail(RTSDF_E_RANGE, "triangles given but no vertices");
    if (bvh_bytes < rtsdf::bvh_bytes(nt))
        return fail(RTSDF_E_SIZE, "bvh buffer %zu < %zu bytes", bvh_bytes, rtsdf::bvh_bytes(nt));
    if (nt > 0 && work_bytes < rtsdf::bvh_work_bytes(nt))
        return fail(RTSDF_E_SIZE, "bvh work %zu < %zu bytes", work_bytes, rtsdf::bvh_work_bytes(nt));
    return device(rtsdf::build_bvh(verts, tris, nt, g, bvh, work, as_stream(stream)), "build_bvh");
}

rtsdf_status rtsdf_reset_accum(float* dmin, uint32_t* hits, uint64_t* argmin, int64_t n, void* stream)
{
    if (n < 0) return fail(RTSDF_E_RANGE, "n < 0");
    if (n > 0 && (!dmin || !hits)) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::reset_accum(dmin, hits, argmin, n, as_stream(stream)), "reset_accum");
}

size_t rtsdf_raysample_work_bytes(int64_t band_capacity, int32_t rays_per_voxel)
{
    return rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel);
}

rtsdf_status rtsdf_raysample(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                             const int32_t* band_count, int64_t band_capacity, int32_t rays_per_voxel,
                             uint64_t rng_key, uint32_t frame, uint32_t obj, float* dmin, uint32_t* hits,
                             uint64_t* argmin, void* work, size_t work_bytes, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!bvh || !band_list || !band_count || !dmin || !hits || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > rtsdf::nvox(g))
        return fail(RTSDF_E_RANGE, "band_capacity outside [0, N]");
    if (obj >= (1u << 24)) return fail(RTSDF_E_RANGE, "obj %u >= 2^24", obj);
    if (work_bytes < rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel))
        return fail(RTSDF_E_SIZE, "raysample work %zu < %zu bytes", work_bytes,
                    rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel));
    return device(rtsdf::raysample(bvh, g, band_list, band_count, band_capacity, rays_per_voxel, rng_key,
                                   frame, obj, dmin, hits, argmin, work, as_stream(stream)),
                  "raysample");
}

rtsdf_status rtsdf_combine(const int32_t* seeds, float* dmin, uint32_t* hits, rtsdf_grid g, int32_t band_vox,
                           float beta, float bias, int32_t mode, float alpha, int32_t first_frame,
                           int32_t consume, float* state, float* fine, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!seeds || !dmin || !hits || !fine) return fail(RTSDF_E_ARG, "NULL pointer");
    if (band_vox < 0 || band_vox > 2048) return fail(RTSDF_E_RANGE, "band_vox %d outside [0, 2048]", band_vox);
    if (mode != RTSDF_ACCUM && mode != RTSDF_DECAY) return fail(RTSDF_E_RANGE, "unknown mode %d", mode);
    if (!std::isfinite(beta) || !std::isfinite(bias)) return fail(RTSDF_E_ARG, "beta and bias must be finite");
    if (mode == RTSDF_DECAY) {
        if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(RTSDF_E_ARG, "alpha outside [0, 1]");
        if (!state) return fail(RTSDF_E_ARG, "DECAY needs a state buffer");
    }
    return device(rtsdf::combine(seeds, dmin, hits, g, band_vox, beta, bias, mode, alpha, first_frame, consume,
                                 state, fine, as_stream(stream)),
                  "combine");
}

rtsdf_status rtsdf_shadow_forward(const float* fine, rtsdf_grid g, rtsdf_shadow s, float* img, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow(s)) return st;
    if (!fine || !img) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::shadow_forward(fine, g, s, img, as_stream(stream)), "shadow_forward");
}

rtsdf_status rtsdf_shadow_backward(const float* fine, rtsdf_grid g, rtsdf_shadow s, const float* grad_img,
                                   float* grad_fine, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow(s)) return st;
    if (!fine || !grad_img || !grad_fine) return fail(RTSDF_E_ARG, "NULL pointer");
    if (fine == grad_fine) return fail(RTSDF_E_ARG, "fine and grad_fine must not alias");
    return device(rtsdf::shadow_backward(fine, g, s, grad_img, grad_fine, as_stream(stream)), "shadow_backward");
}

rtsdf_status rtsdf_backward(const float* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                            const int32_t* band_list, const int32_t* band_count, int64_t band_capacity,
                            const void* bvh, const int32_t* tris, int32_t nv, int32_t nt, rtsdf_grid g,
                            int32_t rays_per_voxel, uint64_t rng_key, uint32_t obj, float* grad_verts,
                            void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (nv < 0 || nt < 0 || nt > (1 << 26)) return fail(RTSDF_E_RANGE, "nv, nt outside [0, 2^26]");
    if (!grad_fine || !hits || !argmin || !band_list || !band_count || !bvh)
        return fail(RTSDF_E_ARG, "NULL pointer");
    if (nt > 0 && (!tris || !grad_verts || nv == 0)) return fail(RTSDF_E_ARG, "tris or grad_verts is NULL");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > rtsdf::nvox(g))
        return fail(RTSDF_E_RANGE, "band_capacity outside [0, N]");
    if (obj >= (1u << 24)) return fail(RTSDF_E_RANGE, "obj %u >= 2^24", obj);
    if (nt == 0) return ok();
    return device(rtsdf::sdf_backward(grad_fine, hits, argmin, band_list, band_count, band_capacity, bvh, tris, g,
                                      rays_per_voxel, rng_key, obj, grad_verts, as_stream(stream)),
                  "backward");
}

}  // extern "C"
