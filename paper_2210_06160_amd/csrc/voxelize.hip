// Conservative voxelization into seed ids (section 2.2).
//
// 1. every grid point <- EMPTY
// 2. one thread per triangle: snap vertices to 1/256 voxel, count the voxels of the
//    triangle's closed-cell range (a candidate box)
// 3. exclusive scan of the counts (64-bit; a big triangle can cover the whole grid)
// 4. one lane per (triangle, candidate voxel), dealt in runs of consecutive candidates so
//    that a lane's triangle changes rarely (see k_candidates): exact integer
//    separating-axis test of the triangle against the closed voxel cube;
//    on overlap the voxel writes its own id.  Every writer of a voxel writes the same
//    value, so the result does not depend on scheduling.
#include "internal.h"

namespace rtsdf {

namespace {

constexpr float kSnapLimit = 524288.0f;  // 2^19 sub-voxels

struct Snapped {
    int32_t X[3][3];  // [vertex][axis], 1/256 voxel units relative to org
    int32_t lo[3], hi[3];
};

__device__ inline int32_t floor_div256(int32_t v) { return v >> 8; }  // arithmetic shift = floor

// Returns false if the triangle is skipped (non-finite or out of range, or no candidate).
__device__ bool snap_triangle(const float* __restrict__ verts, const int32_t* __restrict__ tris,
                              int32_t t, const rtsdf_grid g, Snapped& S)
{
    const int dims[3] = {g.nx, g.ny, g.nz};
    bool ok = true;
    for (int v = 0; v < 3; ++v) {
        const int64_t vi = tris[3 * (int64_t)t + v];
        for (int a = 0; a < 3; ++a) {
            const float q = ((verts[3 * vi + a] - g.org[a]) / g.h) * 256.0f;
            if (!(fabsf(q) <= kSnapLimit)) ok = false;
            S.X[v][a] = ok ? (int32_t)rintf(q) : 0;
        }
    }
    if (!ok) return false;
    for (int a = 0; a < 3; ++a) {
        const int32_t mn = min(min(S.X[0][a], S.X[1][a]), S.X[2][a]);
        const int32_t mx = max(max(S.X[0][a], S.X[1][a]), S.X[2][a]);
        S.lo[a] = max(floor_div256(mn - 1), 0);
        S.hi[a] = min(floor_div256(mx), dims[a] - 1);
        if (S.lo[a] > S.hi[a]) return false;
    }
    return true;
}

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Where triangle t's geometry lives and which grid it is voxelized into.  Single object:
// the arguments themselves.  Batch: t is global; its object (binary search over the
// triangle prefix) supplies the vertex and triangle bases, the grid, and the output buffer
// (`scratch` for objects with an odd JFA pass count, see rtsdf_voxelize_batched).
struct TriSource {
    const float* verts;
    const int32_t* tris;
    int32_t t;
    rtsdf_grid g;
    int32_t* out;
};

template <bool kBatch>
__device__ inline TriSource tri_source(const float* verts, const int32_t* tris, int32_t t, const rtsdf_grid& g,
                                       int32_t* seeds, const char* plan, int32_t nobj, int32_t* scratch)
{
    if (!kBatch) return TriSource{verts, tris, t, g, seeds};
    const BatchView v = batch_view(plan, nobj);
    const BatchObject& ob = v.obj[find_object(v.tri_prefix, nobj, t)];
    return TriSource{verts + 3 * (int64_t)ob.vert_off, tris + 3 * (int64_t)ob.tri_off, t - ob.tri_off, ob.g,
                     (ob.flip ? scratch : seeds) + ob.vox_off};
}

template <bool kBatch>
__global__ void k_count(const float* __restrict__ verts, const int32_t* __restrict__ tris,
                        int32_t nt, const rtsdf_grid g, uint64_t* __restrict__ counts, const char* plan,
                        int32_t nobj)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const TriSource src = tri_source<kBatch>(verts, tris, t, g, nullptr, plan, nobj, nullptr);
    Snapped S;
    uint64_t c = 0;
    if (snap_triangle(src.verts, src.tris, src.t, src.g, S))
        c = (uint64_t)(S.hi[0] - S.lo[0] + 1) * (uint64_t)(S.hi[1] - S.lo[1] + 1) *
            (uint64_t)(S.hi[2] - S.lo[2] + 1);
    counts[t] = c;
}

// Batch: every grid point of every object <- EMPTY in the buffer its seeds start in.
// One kBatchAlign tile per work-group; tiles never straddle objects.
__global__ __launch_bounds__(256) void k_fill_batched(const char* __restrict__ plan, int32_t nobj,
                                                      int32_t* __restrict__ seeds, int32_t* __restrict__ scratch)
{
    const BatchView v = batch_view(plan, nobj);
    const int64_t first = (int64_t)blockIdx.x * kBatchAlign;
    const BatchObject& ob = v.obj[find_object(v.vox_prefix, nobj, first)];
    const int64_t n = (int64_t)ob.g.nx * ob.g.ny * ob.g.nz;
    int32_t* dst = ob.flip ? scratch : seeds;
    for (int64_t i = first + threadIdx.x; i < first + kBatchAlign; i += 256)
        if (i - ob.vox_off < n) dst[i] = RTSDF_EMPTY;
}

// Projection interval test on one axis: [min p, max p] against [-r, r].
__device__ inline bool separated(int64_t p0, int64_t p1, int64_t p2, int64_t r)
{
    const int64_t mn = min(min(p0, p1), p2), mx = max(max(p0, p1), p2);
    return mn > r || mx < -r;
}

__device__ inline int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

// Exact overlap of the closed triangle (sub-voxel coordinates) with the closed cube of
// voxel (i, j, k), i.e. [256 i, 256 i + 256] per axis.
__device__ bool overlaps(const Snapped& S, int32_t i, int32_t j, int32_t k)
{
    const int32_t c[3] = {256 * i + 128, 256 * j + 128, 256 * k + 128};
    int64_t a[3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) a[v][d] = (int64_t)(S.X[v][d] - c[d]);
    // cube face normals
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (separated(a[0][d], a[1][d], a[2][d], 128)) return false;
    // edges
    int64_t f[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f[0][d] = a[1][d] - a[0][d];
        f[1][d] = a[2][d] - a[1][d];
        f[2][d] = a[0][d] - a[2][d];
    }
    // plane normal: every vertex projects to the same value
    const int64_t nx = f[0][1] * f[1][2] - f[0][2] * f[1][1];
    const int64_t ny = f[0][2] * f[1][0] - f[0][0] * f[1][2];
    const int64_t nz = f[0][0] * f[1][1] - f[0][1] * f[1][0];
    {
        const int64_t p = nx * a[0][0] + ny * a[0][1] + nz * a[0][2];
        const int64_t r = 128 * (iabs64(nx) + iabs64(ny) + iabs64(nz));
        if (p > r || p < -r) return false;
    }
    // axis x edge: (0, -fz, fy); axis y edge: (fz, 0, -fx); axis z edge: (-fy, fx, 0)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int64_t fx = f[m][0], fy = f[m][1], fz = f[m][2];
        {
            const int64_t r = 128 * (iabs64(fz) + iabs64(fy));
            if (separated(-fz * a[0][1] + fy * a[0][2], -fz * a[1][1] + fy * a[1][2],
                          -fz * a[2][1] + fy * a[2][2], r))
                return false;
        }
        {
            const int64_t r = 128 * (iabs64(fz) + iabs64(fx));
            if (separated(fz * a[0][0] - fx * a[0][2], fz * a[1][0] - fx * a[1][2],
                          fz * a[2][0] - fx * a[2][2], r))
                return false;
        }
        {
            const int64_t r = 128 * (iabs64(fy) + iabs64(fx));
            if (separated(-fy * a[0][0] + fx * a[0][1], -fy * a[1][0] + fx * a[1][1],
                          -fy * a[2][0] + fx * a[2][1], r))
                return false;
        }
    }
    return true;
}

// Candidates are dealt to lanes in runs of consecutive ones (a wave takes 64 runs at a
// time): a lane's next candidate is in the same triangle unless it crosses the triangle's
// end (triangles hold hundreds of candidates on average at fine resolutions, a few at
// coarse ones), so the triangle is found by a short forward search rather than a full one
// per candidate, and the voxel coordinates advance by one with carries instead of divisions.
// Runs are kCandRun long when there are that many candidates per lane of the launch, and
// shorter when there are fewer, so that every lane still has work.
constexpr int kCandRun = 16;

template <bool kBatch>
__global__ __launch_bounds__(256) void k_candidates(const float* __restrict__ verts,
                                                    const int32_t* __restrict__ tris, int32_t nt,
                                                    const rtsdf_grid g,
                                                    const uint64_t* __restrict__ offsets,
                                                    const uint64_t* __restrict__ total_p,
                                                    int32_t* __restrict__ seeds, const char* plan,
                                                    int32_t nobj, int32_t* __restrict__ scratch)
{
    const uint64_t total = *total_p;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t run = min((uint64_t)kCandRun, max((uint64_t)1, total / (nwaves * 64)));
    const uint64_t chunk = 64 * run;
    int32_t cur = 0;
    uint64_t tri_lo = 1, tri_hi = 0;  // candidates [tri_lo, tri_hi) of triangle cur (none yet)
    Snapped S;
    TriSource src;
    int32_t ex = 1, ey = 1;          // the triangle's candidate box extents on x and y
    int32_t li = 0, lj = 0, lk = 0;  // the candidate's position in the box
    for (uint64_t base = wave * chunk; base < total; base += nwaves * chunk) {
        const uint64_t first = base + (uint64_t)lane * run;
        const uint64_t end = min(first + run, total);
        bool carried = false;  // li, lj, lk hold the position of c - 1 in the same triangle
        for (uint64_t c = first; c < end; ++c) {
            if (c < tri_lo || c >= tri_hi) {
                // triangle owning c: the last t with offsets[t] <= c, searched from the current
                // one (candidates only grow); within a run c has just passed the current
                // triangle's end, so the search gallops forward (steps 1, 2, 4, ..) before
                // bisecting: a few loads for the next triangle, and O(log) ones across long
                // stretches of triangles without candidates
                int32_t lo = cur, hi = nt - 1;
                if (carried) {
                    int32_t step = 1;
                    while (lo + step <= hi && offsets[lo + step] <= c) {
                        lo += step;
                        step <<= 1;
                    }
                    hi = min(hi, lo + step - 1);
                }
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (offsets[mid] <= c) lo = mid;
                    else hi = mid - 1;
                }
                cur = lo;
                tri_lo = offsets[cur];
                tri_hi = cur + 1 < nt ? offsets[cur + 1] : total;
                src = tri_source<kBatch>(verts, tris, cur, g, seeds, plan, nobj, scratch);
                snap_triangle(src.verts, src.tris, src.t, src.g, S);
                ex = S.hi[0] - S.lo[0] + 1;
                ey = S.hi[1] - S.lo[1] + 1;
                carried = false;
            }
            if (carried) {
                if (++li == ex) {
                    li = 0;
                    if (++lj == ey) {
                        lj = 0;
                        ++lk;
                    }
                }
            } else {
                const uint32_t local = (uint32_t)(c - tri_lo);  // a box holds at most 2^30 voxels
                const uint32_t q = local / (uint32_t)ex;
                li = (int32_t)(local - q * (uint32_t)ex);
                lk = (int32_t)(q / (uint32_t)ey);
                lj = (int32_t)q - lk * ey;
            }
            carried = true;
            const int32_t i = S.lo[0] + li, j = S.lo[1] + lj, k = S.lo[2] + lk;
            if (overlaps(S, i, j, k))
                src.out[i + (int64_t)src.g.nx * (j + (int64_t)src.g.ny * k)] = i | (j << 10) | (k << 20);
        }
    }
}

}  // namespace

size_t voxelize_work_bytes(int32_t nt)
{
    const int64_t n = (int64_t)nt + 1;
    return align256((size_t)n * 8) + align256(8) + scan_work_bytes_u64(n);
}

hipError_t voxelize(const float* verts, const int32_t* tris, int32_t nt, const rtsdf_grid& g,
                    int32_t* seeds, void* work, hipStream_t s)
{
    const int64_t N = nvox(g);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(ceil_div(N, 256), 16384)), dim3(256),
                       0, s, seeds, N, (int32_t)RTSDF_EMPTY);
    if (nt == 0) return hipGetLastError();
    char* w = (char*)work;
    uint64_t* offsets = (uint64_t*)w;
    w += align256((size_t)(nt + 1) * 8);
    uint64_t* total = (uint64_t*)w;
    w += align256(8);
    hipLaunchKernelGGL(k_count<false>, dim3((unsigned)ceil_div(nt, 256)), dim3(256), 0, s, verts, tris, nt,
                       g, offsets, nullptr, 0);
    hipError_t e = scan_exclusive_u64(offsets, offsets, nt, total, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_candidates<false>, dim3((unsigned)persistent_groups(256)), dim3(256), 0, s, verts,
                       tris, nt, g, offsets, total, seeds, nullptr, 0, nullptr);
    return hipGetLastError();
}

hipError_t voxelize_batched(const BatchView& hv, const void* dplan, const float* verts, const int32_t* tris,
                            int32_t* seeds, int32_t* scratch, void* work, hipStream_t s)
{
    const int32_t nobj = hv.h->nobj;
    const char* plan = (const char*)dplan;
    const int64_t tiles = hv.h->total_vox / kBatchAlign;
    hipLaunchKernelGGL(k_fill_batched, dim3((unsigned)tiles), dim3(256), 0, s, plan, nobj, seeds, scratch);
    const int32_t nt = (int32_t)hv.h->total_tris;
    if (nt == 0) return hipGetLastError();
    const rtsdf_grid g0 = hv.obj[0].g;  // unused in batch mode
    char* w = (char*)work;
    uint64_t* offsets = (uint64_t*)w;
    w += align256((size_t)(nt + 1) * 8);
    uint64_t* total = (uint64_t*)w;
    w += align256(8);
    hipLaunchKernelGGL(k_count<true>, dim3((unsigned)ceil_div(nt, 256)), dim3(256), 0, s, verts, tris, nt, g0,
                       offsets, plan, nobj);
    hipError_t e = scan_exclusive_u64(offsets, offsets, nt, total, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_candidates<true>, dim3((unsigned)persistent_groups(256)), dim3(256), 0, s, verts, tris,
                       nt, g0, offsets, total, seeds, plan, nobj, scratch);
    return hipGetLastError();
}

}  // namespace rtsdf
