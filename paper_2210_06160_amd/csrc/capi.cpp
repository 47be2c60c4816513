// C ABI of librtsdf.so: host-side validation, then the HIP launchers.  No exception or
// allocation crosses this layer; every failure becomes an rtsdf_status plus a thread-local
// message.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

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

// ---- batched objects: plan construction ------------------------------------------------

size_t batch_work_bytes(const rtsdf::BatchView& v)
{
    size_t w = rtsdf::raysample_work_bytes(0, 1);  // ray-sampling cursors
    w = std::max(w, rtsdf::voxelize_work_bytes((int32_t)v.h->total_tris));
    w = std::max(w, rtsdf::band_batched_work_bytes(v.h->total_vox));
    w = std::max(w, rtsdf::bvh_work_bytes(v.h->total_tris, v.h->total_tiles, v.h->nobj));
    return w;
}

// validates a host plan; fills the view
rtsdf_status check_plan(const void* plan, rtsdf::BatchView& v)
{
    if (!plan) return fail(RTSDF_E_ARG, "plan is NULL");
    const rtsdf::BatchHeader* h = (const rtsdf::BatchHeader*)plan;
    if (h->magic != rtsdf::kBatchMagic || h->nobj < 1 || h->nobj > RTSDF_MAX_OBJECTS || !h->device)
        return fail(RTSDF_E_ARG, "not a batch plan (use the host copy written by rtsdf_batch_plan)");
    v = rtsdf::batch_view(plan, h->nobj);
    return RTSDF_OK;
}

}  // namespace

extern "C" {

size_t rtsdf_batch_plan_bytes(int32_t nobj)
{
    return (nobj < 1 || nobj > RTSDF_MAX_OBJECTS) ? 0 : rtsdf::batch_plan_bytes(nobj);
}

rtsdf_status rtsdf_batch_plan(const rtsdf_object* objs, int32_t nobj, void* plan_host, void* plan_device,
                              size_t plan_bytes, rtsdf_batch_sizes* sizes)
{
    using namespace rtsdf;
    if (!objs || !plan_host || !plan_device || !sizes) return fail(RTSDF_E_ARG, "NULL pointer");
    if (nobj < 1 || nobj > RTSDF_MAX_OBJECTS) return fail(RTSDF_E_RANGE, "nobj %d outside [1, %d]", nobj, RTSDF_MAX_OBJECTS);
    const size_t bytes = batch_plan_bytes(nobj);
    if (plan_bytes < bytes) return fail(RTSDF_E_SIZE, "plan %zu < %zu bytes", plan_bytes, bytes);
    std::vector<char> buf(bytes, 0);
    BatchHeader* h = (BatchHeader*)buf.data();
    BatchView v = batch_view(buf.data(), nobj);
    BatchObject* ob = const_cast<BatchObject*>(v.obj);
    int64_t* vox_prefix = const_cast<int64_t*>(v.vox_prefix);
    int32_t* tri_prefix = const_cast<int32_t*>(v.tri_prefix);
    int32_t* pass_prefix = const_cast<int32_t*>(v.pass_prefix);
    int64_t vox = 0, verts = 0, tris = 0, tiles = 0;
    uint64_t bvh = 0;
    int32_t max_passes = 0;
    for (int32_t o = 0; o < nobj; ++o) {
        const rtsdf_object& in = objs[o];
        if (rtsdf_status st = check_grid(in.g)) {
            char msg[sizeof(g_err)];
            std::snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(st, "object %d: %s", o, msg);
        }
        if (in.nv < 0 || in.nt < 0 || in.nt > rtsdf::kBvhMaxTris)
            return fail(RTSDF_E_RANGE, "object %d: nv %d / nt %d outside range", o, in.nv, in.nt);
        if (in.nt > 0 && in.nv == 0) return fail(RTSDF_E_RANGE, "object %d: triangles but no vertices", o);
        if (in.band_vox < 0 || in.band_vox > 2048) return fail(RTSDF_E_RANGE, "object %d: band_vox outside [0, 2048]", o);
        if (in.extra_passes < 0 || in.extra_passes > 8) return fail(RTSDF_E_RANGE, "object %d: extra_passes outside [0, 8]", o);
        if (!std::isfinite(in.beta) || !std::isfinite(in.bias)) return fail(RTSDF_E_ARG, "object %d: beta/bias not finite", o);
        BatchObject& b = ob[o];
        b.g = in.g;
        b.band_vox = in.band_vox;
        b.vox_off = vox;
        b.bvh_off = (int64_t)bvh;
        b.vert_off = (int32_t)verts;
        b.tri_off = (int32_t)tris;
        b.nv = in.nv;
        b.nt = in.nt;
        const int32_t n = std::max(in.g.nx, std::max(in.g.ny, in.g.nz));
        int32_t k = 1;
        while (k < n) k *= 2;
        b.k0 = std::max(k / 2, 1);
        b.nhalf = 0;
        for (int32_t q = b.k0; q >= 1; q /= 2) ++b.nhalf;
        b.nsteps = b.nhalf + in.extra_passes;
        b.flip = b.nsteps & 1;
        b.beta = in.beta;
        b.bias = in.bias;
        b.tile_off = (int32_t)tiles;
        tiles += ceil_div(in.nt, kBvhSortTile);
        vox_prefix[o] = vox;
        tri_prefix[o] = (int32_t)tris;
        vox += ceil_div(nvox(in.g), kBatchAlign) * kBatchAlign;
        verts += in.nv;
        tris += in.nt;
        bvh += align256(bvh_bytes(in.nt));
        max_passes = std::max(max_passes, b.nsteps);
        if (vox >= ((int64_t)1 << 31) || verts >= ((int64_t)1 << 31) || tris > (1 << 26))
            return fail(RTSDF_E_RANGE, "batch too large: voxels, vertices and triangles must stay below 2^31, 2^31, 2^26");
    }
    vox_prefix[nobj] = vox;
    tri_prefix[nobj] = (int32_t)tris;
    for (int32_t p = 0; p < max_passes; ++p) {
        int32_t* pre = pass_prefix + (int64_t)p * (nobj + 1);
        int64_t acc = 0;
        for (int32_t o = 0; o < nobj; ++o) {
            pre[o] = (int32_t)acc;
            if (p < ob[o].nsteps) acc += jfa_pass_blocks(ob[o].g, jfa_offset(ob[o].k0, ob[o].nhalf, p));
            if (acc >= ((int64_t)1 << 31)) return fail(RTSDF_E_RANGE, "too many JFA work-groups in pass %d", p);
        }
        pre[nobj] = (int32_t)acc;
        h->pass_blocks[p] = (int32_t)acc;
    }
    h->magic = kBatchMagic;
    h->nobj = nobj;
    h->max_passes = max_passes;
    h->total_vox = vox;
    h->total_verts = verts;
    h->total_tris = tris;
    h->bvh_bytes = bvh;
    h->total_tiles = (int32_t)tiles;
    h->plan_bytes = bytes;
    h->device = plan_device;
    std::memcpy(plan_host, buf.data(), bytes);
    sizes->voxels = vox;
    sizes->verts = verts;
    sizes->tris = tris;
    sizes->bvh_bytes = bvh;
    sizes->work_bytes = batch_work_bytes(batch_view(plan_host, nobj));
    sizes->max_passes = max_passes;
    return ok();
}

rtsdf_status rtsdf_batch_upload(const void* plan_host, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan_host, v)) return st;
    hipError_t e = hipMemcpyAsync(const_cast<void*>(v.h->device), plan_host, v.h->plan_bytes, hipMemcpyHostToDevice,
                                  as_stream(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
    return device(e, "batch plan upload");
}

rtsdf_status rtsdf_batch_offsets(const void* plan_host, int32_t o, int64_t* vox_offset, size_t* bvh_offset)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan_host, v)) return st;
    if (o < 0 || o >= v.h->nobj) return fail(RTSDF_E_RANGE, "object %d outside [0, %d)", o, v.h->nobj);
    if (vox_offset) *vox_offset = v.obj[o].vox_off;
    if (bvh_offset) *bvh_offset = (size_t)v.obj[o].bvh_off;
    return ok();
}

rtsdf_status rtsdf_voxelize_batched(const void* plan, const float* verts, const int32_t* tris, int32_t* seeds,
                                    int32_t* scratch, void* work, size_t work_bytes, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!seeds || !scratch || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (seeds == scratch) return fail(RTSDF_E_ARG, "seeds and scratch must not alias");
    if (v.h->total_tris > 0 && (!verts || !tris)) return fail(RTSDF_E_ARG, "verts or tris is NULL");
    if (work_bytes < batch_work_bytes(v)) return fail(RTSDF_E_SIZE, "work %zu < %zu bytes", work_bytes, batch_work_bytes(v));
    return device(rtsdf::voxelize_batched(v, v.h->device, verts, tris, seeds, scratch, work, as_stream(stream)),
                  "voxelize_batched");
}

rtsdf_status rtsdf_jfa_batched(const void* plan, int32_t* seeds, int32_t* scratch, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!seeds || !scratch) return fail(RTSDF_E_ARG, "NULL pointer");
    if (seeds == scratch) return fail(RTSDF_E_ARG, "seeds and scratch must not alias");
    for (int32_t p = 0; p < v.h->max_passes; ++p) {
        hipError_t e = rtsdf::jfa_batched_pass(v, v.h->device, seeds, scratch, p, as_stream(stream));
        if (e != hipSuccess) return device(e, "jfa_batched pass");
    }
    return ok();
}

rtsdf_status rtsdf_band_batched(const void* plan, const int32_t* seeds, int32_t* band_list, int32_t* band_count,
                                void* work, size_t work_bytes, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!seeds || !band_list || !band_count || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (work_bytes < batch_work_bytes(v)) return fail(RTSDF_E_SIZE, "work %zu < %zu bytes", work_bytes, batch_work_bytes(v));
    return device(rtsdf::band_batched(v, v.h->device, seeds, band_list, band_count, work, as_stream(stream)),
                  "band_batched");
}

rtsdf_status rtsdf_build_bvh_batched(const void* plan, const float* verts, const int32_t* tris, int32_t method,
                                     void* bvh, size_t bvh_bytes, void* work, size_t work_bytes, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!bvh || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (method != RTSDF_BVH_LBVH && method != RTSDF_BVH_PLOC) return fail(RTSDF_E_RANGE, "unknown method %d", method);
    if (v.h->total_tris > 0 && (!verts || !tris)) return fail(RTSDF_E_ARG, "verts or tris is NULL");
    if (bvh_bytes < v.h->bvh_bytes) return fail(RTSDF_E_SIZE, "bvh %zu < %zu bytes", bvh_bytes, (size_t)v.h->bvh_bytes);
    if (work_bytes < batch_work_bytes(v)) return fail(RTSDF_E_SIZE, "work %zu < %zu bytes", work_bytes, batch_work_bytes(v));
    return device(rtsdf::build_bvh_batched(v, v.h->device, verts, tris, bvh, work, method, as_stream(stream)),
                  "build_bvh_batched");
}

rtsdf_status rtsdf_raysample_batched(const void* plan, const void* bvh, const int32_t* band_list,
                                     const int32_t* band_count, int64_t band_capacity, int32_t rays_per_voxel,
                                     uint64_t rng_key, uint32_t frame, float* dmin, uint32_t* hits, uint64_t* argmin,
                                     void* work, size_t work_bytes, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!bvh || !band_list || !band_count || !dmin || !hits || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > v.h->total_vox) return fail(RTSDF_E_RANGE, "band_capacity outside [0, voxels]");
    if (v.h->nobj > (1 << 24)) return fail(RTSDF_E_RANGE, "object index must fit 24 bits");
    if (work_bytes < batch_work_bytes(v)) return fail(RTSDF_E_SIZE, "work %zu < %zu bytes", work_bytes, batch_work_bytes(v));
    return device(rtsdf::raysample_batched(v, v.h->device, bvh, band_list, band_count, band_capacity, rays_per_voxel,
                                           rng_key, frame, dmin, hits, argmin, work, as_stream(stream)),
                  "raysample_batched");
}

rtsdf_status rtsdf_combine_batched(const void* plan, const int32_t* seeds, const float* dmin, const uint32_t* hits,
                                   float* fine, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!seeds || !dmin || !hits || !fine) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::combine_batched(v, v.h->device, seeds, dmin, hits, fine, as_stream(stream)), "combine_batched");
}

rtsdf_status rtsdf_backward_batched(const void* plan, const float* grad_fine, const uint32_t* hits,
                                    const uint64_t* argmin, const int32_t* band_list, const int32_t* band_count,
                                    int64_t band_capacity, const void* bvh, const int32_t* tris, int32_t rays_per_voxel,
                                    uint64_t rng_key, float* grad_verts, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (!grad_fine || !hits || !argmin || !band_list || !band_count || !bvh) return fail(RTSDF_E_ARG, "NULL pointer");
    if (v.h->total_tris > 0 && (!tris || !grad_verts)) return fail(RTSDF_E_ARG, "tris or grad_verts is NULL");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > v.h->total_vox) return fail(RTSDF_E_RANGE, "band_capacity outside [0, voxels]");
    return device(rtsdf::sdf_backward_batched(v, v.h->device, grad_fine, hits, argmin, band_list, band_count,
                                              band_capacity, bvh, tris, rays_per_voxel, rng_key, grad_verts,
                                              as_stream(stream)),
                  "backward_batched");
}

const char* rtsdf_last_error(void) { return g_err; }

int32_t rtsdf_abi_version(void) { return 2; }

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
        hipError_t e = rtsdf::jfa_pass(a, b, g, steps[i], i == 0, i + 1 == nsteps, as_stream(stream));
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
                             rtsdf_grid g, int32_t method, void* bvh, size_t bvh_bytes, void* work,
                             size_t work_bytes, void* stream)
{
    if (method != RTSDF_BVH_LBVH && method != RTSDF_BVH_PLOC) return fail(RTSDF_E_RANGE, "unknown method %d", method);
    if (rtsdf_status st = check_grid(g)) return st;
    if (nv < 0 || nt < 0 || nt > rtsdf::kBvhMaxTris) return fail(RTSDF_E_RANGE, "nt %d outside [0, 2^26]", nt);
    if (!bvh) return fail(RTSDF_E_ARG, "bvh is NULL");
    if (nt > 0 && (!verts || !tris || !work)) return fail(RTSDF_E_ARG, "verts, tris or work is NULL");
    if (nt > 0 && nv == 0) return fail(RTSDF_E_RANGE, "triangles given but no vertices");
    if (bvh_bytes < rtsdf::bvh_bytes(nt))
        return fail(RTSDF_E_SIZE, "bvh buffer %zu < %zu bytes", bvh_bytes, rtsdf::bvh_bytes(nt));
    if (nt > 0 && work_bytes < rtsdf::bvh_work_bytes(nt))
        return fail(RTSDF_E_SIZE, "bvh work %zu < %zu bytes", work_bytes, rtsdf::bvh_work_bytes(nt));
    return device(rtsdf::build_bvh(verts, tris, nt, g, bvh, work, method, as_stream(stream)), "build_bvh");
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
                                   frame, nullptr, obj, dmin, hits, argmin, work, as_stream(stream)),
                  "raysample");
}

rtsdf_status rtsdf_raysample_frame_device(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                                          const int32_t* band_count, int64_t band_capacity, int32_t rays_per_voxel,
                                          uint64_t rng_key, const uint32_t* frame, uint32_t obj, float* dmin,
                                          uint32_t* hits, uint64_t* argmin, void* work, size_t work_bytes,
                                          void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!bvh || !band_list || !band_count || !frame || !dmin || !hits || !work)
        return fail(RTSDF_E_ARG, "NULL pointer");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > rtsdf::nvox(g))
        return fail(RTSDF_E_RANGE, "band_capacity outside [0, N]");
    if (obj >= (1u << 24)) return fail(RTSDF_E_RANGE, "obj %u >= 2^24", obj);
    if (work_bytes < rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel))
        return fail(RTSDF_E_SIZE, "raysample work %zu < %zu bytes", work_bytes,
                    rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel));
    return device(rtsdf::raysample(bvh, g, band_list, band_count, band_capacity, rays_per_voxel, rng_key, 0u, frame,
                                   obj, dmin, hits, argmin, work, as_stream(stream)),
                  "raysample_frame_device");
}

rtsdf_status rtsdf_raysample_noalloc(const void* bvh, rtsdf_grid g, const int32_t* band_list,
                                     const int32_t* band_count, int64_t band_capacity, int32_t rays_per_voxel,
                                     uint64_t rng_key, uint32_t frame, uint32_t obj, float* dmin, uint32_t* hits,
                                     uint64_t* argmin, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (!bvh || !band_list || !band_count || !dmin || !hits) return fail(RTSDF_E_ARG, "NULL pointer");
    if (rays_per_voxel < 1 || rays_per_voxel > RTSDF_MAX_RAYS)
        return fail(RTSDF_E_RANGE, "rays_per_voxel %d outside [1, %d]", rays_per_voxel, RTSDF_MAX_RAYS);
    if (band_capacity < 0 || band_capacity > rtsdf::nvox(g))
        return fail(RTSDF_E_RANGE, "band_capacity outside [0, N]");
    if (obj >= (1u << 24)) return fail(RTSDF_E_RANGE, "obj %u >= 2^24", obj);
    const size_t need = rtsdf::raysample_work_bytes(band_capacity, rays_per_voxel);
    if (need > rtsdf::raysample_scratch_bytes())
        return fail(RTSDF_E_SIZE, "raysample work %zu bytes exceeds the static scratch of %zu bytes", need,
                    rtsdf::raysample_scratch_bytes());
    void* scratch = nullptr;
    if (rtsdf_status st = device(rtsdf::raysample_scratch(&scratch), "raysample scratch address")) return st;
    return device(rtsdf::raysample(bvh, g, band_list, band_count, band_capacity, rays_per_voxel, rng_key, frame,
                                   nullptr, obj, dmin, hits, argmin, scratch, as_stream(stream)),
                  "raysample_noalloc");
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

rtsdf_status rtsdf_refine_grid(rtsdf_grid coarse, int32_t ratio, rtsdf_grid* fine)
{
    if (rtsdf_status st = check_grid(coarse)) return st;
    if (!fine) return fail(RTSDF_E_ARG, "fine is NULL");
    if (ratio < 1 || ratio > RTSDF_MAX_DIM) return fail(RTSDF_E_RANGE, "ratio %d outside [1, %d]", ratio, RTSDF_MAX_DIM);
    const int64_t fx = (int64_t)coarse.nx * ratio, fy = (int64_t)coarse.ny * ratio, fz = (int64_t)coarse.nz * ratio;
    if (fx > RTSDF_MAX_DIM || fy > RTSDF_MAX_DIM || fz > RTSDF_MAX_DIM)
        return fail(RTSDF_E_RANGE, "refined grid %lld x %lld x %lld exceeds %d per axis", (long long)fx,
                    (long long)fy, (long long)fz, RTSDF_MAX_DIM);
    rtsdf_grid f = coarse;
    f.nx = (int32_t)fx;
    f.ny = (int32_t)fy;
    f.nz = (int32_t)fz;
    f.h = coarse.h / (float)ratio;
    *fine = f;
    return ok();
}

size_t rtsdf_band_refined_work_bytes(rtsdf_grid coarse, int32_t ratio)
{
    rtsdf_grid f;
    if (rtsdf_refine_grid(coarse, ratio, &f) != RTSDF_OK) return 0;
    return rtsdf::band_refined_work_bytes(coarse, ratio);
}

rtsdf_status rtsdf_band_refined(const int32_t* seeds, rtsdf_grid coarse, int32_t ratio, int32_t band_vox,
                                int32_t* band_list, int32_t* band_count, void* work, size_t work_bytes,
                                void* stream)
{
    rtsdf_grid f;
    if (rtsdf_status st = rtsdf_refine_grid(coarse, ratio, &f)) return st;
    if (!seeds || !band_list || !band_count || !work) return fail(RTSDF_E_ARG, "NULL pointer");
    if (band_vox < 0 || band_vox > 2048) return fail(RTSDF_E_RANGE, "band_vox %d outside [0, 2048]", band_vox);
    const size_t need = rtsdf::band_refined_work_bytes(coarse, ratio);
    if (work_bytes < need) return fail(RTSDF_E_SIZE, "band work %zu < %zu bytes", work_bytes, need);
    return device(rtsdf::band_refined(seeds, coarse, ratio, band_vox, band_list, band_count, work, as_stream(stream)),
                  "band_refined");
}

rtsdf_status rtsdf_combine_refined(const int32_t* seeds, float* dmin, uint32_t* hits, rtsdf_grid coarse,
                                   int32_t ratio, int32_t band_vox, float beta, float bias, int32_t mode,
                                   float alpha, int32_t first_frame, int32_t consume, float* state,
                                   float* fine, void* stream)
{
    rtsdf_grid f;
    if (rtsdf_status st = rtsdf_refine_grid(coarse, ratio, &f)) return st;
    if (!seeds || !dmin || !hits || !fine) return fail(RTSDF_E_ARG, "NULL pointer");
    if (band_vox < 0 || band_vox > 2048) return fail(RTSDF_E_RANGE, "band_vox %d outside [0, 2048]", band_vox);
    if (mode != RTSDF_ACCUM && mode != RTSDF_DECAY) return fail(RTSDF_E_RANGE, "unknown mode %d", mode);
    if (!std::isfinite(beta) || !std::isfinite(bias)) return fail(RTSDF_E_ARG, "beta and bias must be finite");
    if (mode == RTSDF_DECAY) {
        if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(RTSDF_E_ARG, "alpha outside [0, 1]");
        if (!state) return fail(RTSDF_E_ARG, "DECAY needs a state buffer");
    }
    return device(rtsdf::combine_refined(seeds, dmin, hits, coarse, ratio, band_vox, beta, bias, mode, alpha,
                                         first_frame, consume, state, fine, as_stream(stream)),
                  "combine_refined");
}

rtsdf_status rtsdf_shadow_forward(const float* fine, rtsdf_grid g, rtsdf_shadow s, float* img, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow(s)) return st;
    const bool empty = s.width == 0 || s.height == 0;
    if (!fine || (!img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::shadow_forward(fine, g, s, img, as_stream(stream)), "shadow_forward");
}

rtsdf_status rtsdf_shadow_backward(const float* fine, rtsdf_grid g, rtsdf_shadow s, const float* grad_img,
                                   float* grad_fine, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow(s)) return st;
    const bool empty = s.width == 0 || s.height == 0;
    if (!fine || !grad_fine || (!grad_img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    if (fine == grad_fine) return fail(RTSDF_E_ARG, "fine and grad_fine must not alias");
    return device(rtsdf::shadow_backward(fine, g, s, grad_img, grad_fine, as_stream(stream)), "shadow_backward");
}

namespace {

rtsdf_status check_shadow_ex(const rtsdf_shadow_ex* s)
{
    if (!s) return fail(RTSDF_E_ARG, "shadow parameters are NULL");
    if (rtsdf_status st = check_shadow(s->base)) return st;
    if (s->nlights < 1 || s->nlights > RTSDF_MAX_LIGHTS)
        return fail(RTSDF_E_RANGE, "nlights %d outside [1, %d]", s->nlights, RTSDF_MAX_LIGHTS);
    for (int l = 0; l < s->nlights; ++l)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(s->lights[l][a])) return fail(RTSDF_E_ARG, "light %d is not finite", l);
    if (!std::isfinite(s->jitter) || s->jitter < 0.0f) return fail(RTSDF_E_ARG, "jitter must be finite and >= 0");
    return RTSDF_OK;
}

}  // namespace

rtsdf_status rtsdf_shadow_forward_ex(const float* fine, rtsdf_grid g, const rtsdf_shadow_ex* s, float* img,
                                     void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow_ex(s)) return st;
    const bool empty = s->base.width == 0 || s->base.height == 0;
    if (!fine || (!img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::shadow_forward_ex(fine, g, *s, img, as_stream(stream)), "shadow_forward_ex");
}

rtsdf_status rtsdf_shadow_backward_ex(const float* fine, rtsdf_grid g, const rtsdf_shadow_ex* s,
                                      const float* grad_img, float* grad_fine, void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (rtsdf_status st = check_shadow_ex(s)) return st;
    const bool empty = s->base.width == 0 || s->base.height == 0;
    if (!fine || !grad_fine || (!grad_img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    if (fine == grad_fine) return fail(RTSDF_E_ARG, "fine and grad_fine must not alias");
    return device(rtsdf::shadow_backward_ex(fine, g, *s, grad_img, grad_fine, as_stream(stream)),
                  "shadow_backward_ex");
}

rtsdf_status rtsdf_clipmap_levels(const float* camera, float h0, int32_t n, int32_t levels, rtsdf_grid* grids)
{
    if (!camera || !grids) return fail(RTSDF_E_ARG, "NULL pointer");
    if (!std::isfinite(h0) || !(h0 > 0.0f)) return fail(RTSDF_E_ARG, "h0 must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(camera[a])) return fail(RTSDF_E_ARG, "camera must be finite");
    if (n < 4 || n > RTSDF_MAX_DIM || (n & 1)) return fail(RTSDF_E_RANGE, "n %d not even in [4, %d]", n, RTSDF_MAX_DIM);
    if (levels < 1 || levels > RTSDF_MAX_CLIP_LEVELS)
        return fail(RTSDF_E_RANGE, "levels %d outside [1, %d]", levels, RTSDF_MAX_CLIP_LEVELS);
    for (int32_t l = 0; l < levels; ++l) {
        rtsdf_grid& g = grids[l];
        g.nx = g.ny = g.nz = n;
        g.h = std::ldexp(h0, l);
        if (!std::isfinite(g.h)) return fail(RTSDF_E_ARG, "level %d voxel size overflows", l);
        for (int a = 0; a < 3; ++a) g.org[a] = (std::floor(camera[a] / g.h) - (float)(n / 2)) * g.h;
    }
    return ok();
}

namespace {

rtsdf_status check_clip(const void* plan, rtsdf::BatchView& v)
{
    if (rtsdf_status st = check_plan(plan, v)) return st;
    if (v.h->nobj < 1 || v.h->nobj > RTSDF_MAX_CLIP_LEVELS)
        return fail(RTSDF_E_RANGE, "a clip map has 1 to %d levels, the plan has %d objects", RTSDF_MAX_CLIP_LEVELS,
                    v.h->nobj);
    return RTSDF_OK;
}

}  // namespace

rtsdf_status rtsdf_clipmap_sample(const void* plan, const float* fine, const float* points, int64_t n, float* values,
                                  int32_t* levels, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_clip(plan, v)) return st;
    if (n < 0) return fail(RTSDF_E_RANGE, "n < 0");
    if (n > 0 && (!fine || !points || !values)) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::clip_sample(v, fine, points, n, values, levels, as_stream(stream)), "clipmap_sample");
}

rtsdf_status rtsdf_shadow_forward_clip(const void* plan, const float* fine, const rtsdf_shadow_ex* s, float* img,
                                       void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_clip(plan, v)) return st;
    if (rtsdf_status st = check_shadow_ex(s)) return st;
    const bool empty = s->base.width == 0 || s->base.height == 0;
    if (!fine || (!img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    return device(rtsdf::shadow_forward_clip(v, fine, *s, img, as_stream(stream)), "shadow_forward_clip");
}

rtsdf_status rtsdf_shadow_backward_clip(const void* plan, const float* fine, const rtsdf_shadow_ex* s,
                                        const float* grad_img, float* grad_fine, void* stream)
{
    rtsdf::BatchView v;
    if (rtsdf_status st = check_clip(plan, v)) return st;
    if (rtsdf_status st = check_shadow_ex(s)) return st;
    const bool empty = s->base.width == 0 || s->base.height == 0;
    if (!fine || !grad_fine || (!grad_img && !empty)) return fail(RTSDF_E_ARG, "NULL pointer");
    if (fine == grad_fine) return fail(RTSDF_E_ARG, "fine and grad_fine must not alias");
    return device(rtsdf::shadow_backward_clip(v, fine, *s, grad_img, grad_fine, as_stream(stream)),
                  "shadow_backward_clip");
}

rtsdf_status rtsdf_backward(const float* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                            const int32_t* band_list, const int32_t* band_count, int64_t band_capacity,
                            const void* bvh, const int32_t* tris, int32_t nv, int32_t nt, rtsdf_grid g,
                            int32_t rays_per_voxel, uint64_t rng_key, uint32_t obj, float* grad_verts,
                            void* stream)
{
    if (rtsdf_status st = check_grid(g)) return st;
    if (nv < 0 || nt < 0 || nt > rtsdf::kBvhMaxTris) return fail(RTSDF_E_RANGE, "nv, nt outside [0, 2^26]");
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
