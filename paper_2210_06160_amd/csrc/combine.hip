// Ray mask compaction (section 2.3), accumulator reset, and the coarse/fine combination
// (section 2.1 running minimum, section 2.5.1 Eq. 1 decay, section 2.5.3 bias).
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kBandThreads = 256;
constexpr int kBandItems = 16;  // slices of kBandThreads consecutive voxels per work-group
constexpr int kBandTile = kBandThreads * kBandItems;
constexpr int kBandWaves = kBandThreads / kWave;

// v / r for a fine coordinate v < 1024 and a refinement ratio r in [1, 1024]:
// trunc(v RN(1/r) + RN(0.5/r)) in binary32 with one rounding is exact over that whole range
// (checked exhaustively on the host), and costs a few instructions instead of an integer
// division.
struct ParentOf {
    float inv, half;
    __device__ explicit ParentOf(int32_t r) : inv(1.0f / (float)r), half(0.5f * inv) {}
    __device__ int32_t operator()(int32_t v) const { return (int32_t)fmaf((float)v, inv, half); }
};

__device__ inline int32_t seed_d2(int32_t s, int32_t x, int32_t y, int32_t z)
{
    const int32_t dx = (s & 1023) - x, dy = ((s >> 10) & 1023) - y, dz = ((s >> 20) & 1023) - z;
    return dx * dx + dy * dy + dz * dz;
}

// The grid a mask work-group scans.  Single object: the arguments (a refined grid also
// names its coarse dimensions and ratio).  Batch: the object that owns the work-group's
// tile (tiles are kBatchAlign = kBandTile voxels and never straddle objects); `base` is
// added to the listed indices.
struct BandGrid {
    const int32_t* seeds;
    int64_t N, tile, base;  // points of the grid, its first point of this tile, list index offset
    int32_t nx, ny, b2;
};

struct BandArgs {
    const int32_t* seeds;
    int64_t N;               // points of the masked grid
    int32_t nx, ny, b2;      // masked grid
    int32_t r, cnx, cny;     // refinement ratio and coarse dimensions (refined mask only)
};

template <bool kBatch>
__device__ inline BandGrid band_grid(const BandArgs& a, const char* plan, int32_t nobj)
{
    const int64_t tile = (int64_t)blockIdx.x * kBandTile;
    if (!kBatch) return BandGrid{a.seeds, a.N, tile, 0, a.nx, a.ny, a.b2};
    const BatchView v = batch_view(plan, nobj);
    const BatchObject& ob = v.obj[find_object(v.vox_prefix, nobj, tile)];
    return BandGrid{a.seeds + ob.vox_off, nvox(ob.g), tile - ob.vox_off, ob.vox_off, ob.g.nx, ob.g.ny,
                    ob.band_vox * ob.band_vox};
}

// (x, y, z) of a point of an nx x ny plane grid advanced by kBandThreads points: the step
// split into planes, rows and columns once, then added with carries (no division per step)
struct SliceStep {
    int32_t nx, ny, dx, dy, dz;
    __device__ SliceStep(int32_t nx_, int32_t ny_) : nx(nx_), ny(ny_)
    {
        const int32_t plane = nx * ny;  // at most 2^20
        dz = kBandThreads / plane;
        const int32_t rem = kBandThreads - dz * plane;
        dy = rem / nx;
        dx = rem - dy * nx;
    }
    __device__ void advance(int32_t& x, int32_t& y, int32_t& z) const
    {
        x += dx;
        const int32_t cx = x >= nx ? 1 : 0;  // dx < nx, so one carry at most
        x -= cx * nx;
        y += dy + cx;
        const int32_t cy = y >= ny ? 1 : 0;  // dy < ny
        y -= cy * ny;
        z += dz + cy;
    }
};

// The mask flags of one work-group's tile as wave ballots: slice i covers the kBandThreads
// points tile + i kBandThreads ..; lane t of wave w flags point tile + i kBandThreads +
// w 64 + t.  Loads are consecutive across the work-group, and all kBandItems of a thread
// are issued before the first is tested, so they are in flight together.  (nx, ny) are
// the dimensions of the masked grid; with kRef it is refined by r over a coarse grid of
// (cnx, cny) columns and rows and point (x, y, z) takes the flag of its parent
// (x / r, y / r, z / r).
template <bool kRef>
__device__ void band_ballots(const BandGrid& bg, int32_t r, int32_t cnx, int32_t cny, uint64_t* ballot)
{
    const ParentOf parent(r);
    const int64_t p0 = bg.tile + threadIdx.x;
    const SliceStep st(bg.nx, bg.ny);
    const int64_t row = p0 / bg.nx;
    const int32_t x0 = (int32_t)(p0 - row * bg.nx), y0 = (int32_t)(row % bg.ny), z0 = (int32_t)(row / bg.ny);
    int32_t s[kBandItems];
    if (!kRef) {
#pragma unroll
        for (int i = 0; i < kBandItems; ++i) {
            const int64_t p = p0 + (int64_t)i * kBandThreads;
            s[i] = p < bg.N ? bg.seeds[p] : RTSDF_EMPTY;
        }
    } else {
        int32_t x = x0, y = y0, z = z0;
#pragma unroll
        for (int i = 0; i < kBandItems; ++i) {
            const int64_t p = p0 + (int64_t)i * kBandThreads;
            s[i] = p < bg.N ? bg.seeds[parent(x) + (int64_t)cnx * (parent(y) + (int64_t)cny * parent(z))]
                            : RTSDF_EMPTY;
            st.advance(x, y, z);
        }
    }
    int32_t x = x0, y = y0, z = z0;
#pragma unroll
    for (int i = 0; i < kBandItems; ++i) {
        const int32_t cx = kRef ? parent(x) : x, cy = kRef ? parent(y) : y, cz = kRef ? parent(z) : z;
        // points past the grid's end loaded EMPTY
        const bool in = s[i] != RTSDF_EMPTY && seed_d2(s[i], cx, cy, cz) <= bg.b2;
        ballot[i] = __ballot(in);
        st.advance(x, y, z);
    }
}

template <bool kBatch, bool kRef>
__global__ __launch_bounds__(kBandThreads) void k_band_count(const BandArgs a, uint32_t* __restrict__ counts,
                                                             uint64_t* __restrict__ ballots, const char* plan,
                                                             int32_t nobj)
{
    __shared__ uint32_t part[kBandWaves];
    const BandGrid bg = band_grid<kBatch>(a, plan, nobj);
    uint64_t b[kBandItems];
    band_ballots<kRef>(bg, a.r, a.cnx, a.cny, b);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kBandItems; ++i) c += (uint32_t)__popcll(b[i]);
    // lane i of each wave stores the wave's slice-i ballot: [tile][slice][wave]
    uint64_t mine = 0;
#pragma unroll
    for (int i = 0; i < kBandItems; ++i) mine = lane == i ? b[i] : mine;
    if (lane < kBandItems) ballots[((int64_t)blockIdx.x * kBandItems + lane) * kBandWaves + wave] = mine;
    if (lane == 0) part[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBandWaves; ++w) t += part[w];
        counts[blockIdx.x] = t;
    }
}

// Lists the tile's flagged points in increasing order from the stored ballots: slice i's
// points follow slices 0 .. i-1, and within a slice wave w's follow waves 0 .. w-1.
template <bool kBatch>
__global__ __launch_bounds__(kBandThreads) void k_band_write(const BandArgs a,
                                                             const uint32_t* __restrict__ offsets,
                                                             const uint64_t* __restrict__ ballots,
                                                             int32_t* __restrict__ list, const char* plan,
                                                             int32_t nobj)
{
    static_assert(kBandItems * kBandWaves == kWave, "one ballot per lane of the first wave");
    __shared__ uint32_t pre[kWave];      // list position of each (slice, wave)
    __shared__ uint64_t bal[kWave];
    const int64_t tile = (int64_t)blockIdx.x * kBandTile;
    const uint64_t* tb = ballots + (int64_t)blockIdx.x * kBandItems * kBandWaves;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (wave == 0) {  // exclusive scan of the 64 ballots' counts, one per lane
        const uint64_t bw = tb[lane];
        const uint32_t n = (uint32_t)__popcll(bw);
        uint32_t incl = n;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d);
            if (lane >= d) incl += o;
        }
        pre[lane] = offsets[blockIdx.x] + incl - n;
        bal[lane] = bw;
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < kBandItems; ++i) {
        const uint64_t bw = bal[i * kBandWaves + wave];
        if ((bw >> lane) & 1ull)
            list[pre[i * kBandWaves + wave] + (uint32_t)__popcll(bw & below)] =
                (int32_t)(tile + (int64_t)i * kBandThreads + threadIdx.x);  // batch: the concatenated index
    }
}

__global__ void k_store_count(const uint32_t* __restrict__ total, int32_t* __restrict__ count)
{
    *count = (int32_t)*total;
}

__global__ void k_reset(float* __restrict__ dmin, uint32_t* __restrict__ hits,
                        uint64_t* __restrict__ argmin, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        dmin[i] = __int_as_float(0x7f800000);
        hits[i] = 0u;
        if (argmin) argmin[i] = ~0ull;
    }
}

// One thread per point of the combined grid.  g is the jump-flooded grid; the combined
// grid has r times its points per axis (kRef) or is g itself (r = 1), and each of its
// points takes the coarse distance, inside flag and band test of the coarse point it lies in.
template <int MODE, bool kRef>
__global__ __launch_bounds__(256) void k_combine(const int32_t* __restrict__ seeds,
                                                 float* __restrict__ dmin,
                                                 uint32_t* __restrict__ hits, const rtsdf_grid g, int32_t r,
                                                 int32_t b2, float beta, float bias, float alpha,
                                                 float one_minus_alpha, int32_t first_frame,
                                                 int32_t consume, float* __restrict__ state,
                                                 float* __restrict__ fine)
{
    const int32_t fnx = kRef ? g.nx * r : g.nx, fny = kRef ? g.ny * r : g.ny;
    const int32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int32_t y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int32_t z = blockIdx.z;
    if (x >= fnx || y >= fny) return;
    const int64_t p = x + (int64_t)fnx * (y + (int64_t)fny * z);
    const ParentOf parent(r);
    const int32_t cx = kRef ? parent(x) : x, cy = kRef ? parent(y) : y, cz = kRef ? parent(z) : z;
    const int32_t s = seeds[cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz)];
    float u = __int_as_float(0x7f800000);
    bool inband = false;
    if (s != RTSDF_EMPTY) {
        const int32_t d2 = seed_d2(s, cx, cy, cz);
        u = g.h * sqrtf((float)d2);
        inband = d2 <= b2;
    }
    const float c = u - beta;
    const uint32_t hc = hits[p];
    const uint32_t front = hc & 0xFFFFu, back = hc >> 16;
    float v;
    if (MODE == RTSDF_ACCUM) {
        if (inband && hc != 0u) {
            const float d = dmin[p];
            v = back > front ? -d : d;
        } else {
            v = c;
        }
    } else {
        if (!inband) {
            state[p] = u;
            v = c;
        } else {
            const float prev = state[p];
            float mprev = u, sprev = 1.0f;
            if (!first_frame && isfinite(prev)) {
                mprev = fabsf(prev);
                sprev = signbit(prev) ? -1.0f : 1.0f;
            }
            const float blend = alpha * mprev + one_minus_alpha * u;
            const float r = hc != 0u ? dmin[p] : __int_as_float(0x7f800000);
            const float m = blend < r ? blend : r;
            const float sg = back > front ? -1.0f : (front > back ? 1.0f : sprev);
            v = copysignf(m, sg);
            state[p] = v;
        }
    }
    fine[p] = v - bias;
    if (consume && hc != 0u) {
        dmin[p] = __int_as_float(0x7f800000);
        hits[p] = 0u;
    }
}

// Batch, running minimum only: one kBatchAlign tile per work-group, 16 voxels per thread
// at a stride of 256 (coalesced), coordinates from the object-local index.
__global__ __launch_bounds__(256) void k_combine_batched(const char* __restrict__ plan, int32_t nobj,
                                                         const int32_t* __restrict__ seeds,
                                                         const float* __restrict__ dmin,
                                                         const uint32_t* __restrict__ hits, float* __restrict__ fine)
{
    const BatchView v = batch_view(plan, nobj);
    const int64_t tile = (int64_t)blockIdx.x * kBatchAlign;
    const BatchObject& ob = v.obj[find_object(v.vox_prefix, nobj, tile)];
    const uint32_t nx = (uint32_t)ob.g.nx, ny = (uint32_t)ob.g.ny;
    const uint32_t n = (uint32_t)nvox(ob.g);
    const int32_t b2 = ob.band_vox * ob.band_vox;
    const float h = ob.g.h, beta = ob.beta, bias = ob.bias;
    const uint32_t local0 = (uint32_t)(tile - ob.vox_off);
#pragma unroll 4
    for (int i = 0; i < (int)(kBatchAlign / 256); ++i) {
        const uint32_t local = local0 + (uint32_t)(i * 256) + threadIdx.x;
        if (local >= n) break;
        const uint32_t row = local / nx;
        const int32_t x = (int32_t)(local - row * nx), y = (int32_t)(row % ny), z = (int32_t)(row / ny);
        const int64_t p = ob.vox_off + local;
        const int32_t sd = seeds[p];
        float u = __int_as_float(0x7f800000);
        bool inband = false;
        if (sd != RTSDF_EMPTY) {
            const int32_t d2 = seed_d2(sd, x, y, z);
            u = h * sqrtf((float)d2);
            inband = d2 <= b2;
        }
        const uint32_t hc = hits[p];
        float val = u - beta;
        if (inband && hc != 0u) {
            const float d = dmin[p];
            val = (hc >> 16) > (hc & 0xFFFFu) ? -d : d;
        }
        fine[p] = val - bias;
    }
}

}  // namespace

namespace {

size_t band_work_points(int64_t N)
{
    const int64_t nb = ceil_div(N, kBandTile);
    return align256((size_t)nb * 4) + align256((size_t)nb * kBandItems * kBandWaves * 8) + align256(4) +
           scan_work_bytes_u32(nb);
}

// count, scan, write: the mask list of the grid `a` describes (or of a batch when `plan`)
template <bool kBatch, bool kRef>
hipError_t band_launch(const BandArgs& a, int64_t nb, const char* plan, int32_t nobj, int32_t* list,
                       int32_t* count, void* work, hipStream_t s)
{
    char* w = (char*)work;
    uint32_t* counts = (uint32_t*)w;
    w += align256((size_t)nb * 4);
    uint64_t* ballots = (uint64_t*)w;
    w += align256((size_t)nb * kBandItems * kBandWaves * 8);
    uint32_t* total = (uint32_t*)w;
    w += align256(4);
    hipLaunchKernelGGL((k_band_count<kBatch, kRef>), dim3((unsigned)nb), dim3(kBandThreads), 0, s, a, counts,
                       ballots, plan, nobj);
    hipError_t e = scan_exclusive_u32(counts, counts, nb, total, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_band_write<kBatch>), dim3((unsigned)nb), dim3(kBandThreads), 0, s, a,
                       (const uint32_t*)counts, (const uint64_t*)ballots, list, plan, nobj);
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, (const uint32_t*)total, count);
    return hipGetLastError();
}

}  // namespace

size_t band_work_bytes(const rtsdf_grid& g) { return band_work_points(nvox(g)); }

size_t band_refined_work_bytes(const rtsdf_grid& coarse, int32_t r)
{
    return band_work_points(nvox(coarse) * r * r * r);
}

hipError_t band(const int32_t* seeds, const rtsdf_grid& g, int32_t band_vox, int32_t* list,
                int32_t* count, void* work, hipStream_t s)
{
    const BandArgs a{seeds, nvox(g), g.nx, g.ny, band_vox * band_vox, 1, g.nx, g.ny};
    return band_launch<false, false>(a, ceil_div(a.N, kBandTile), nullptr, 0, list, count, work, s);
}

hipError_t band_refined(const int32_t* seeds, const rtsdf_grid& coarse, int32_t r, int32_t band_vox,
                        int32_t* list, int32_t* count, void* work, hipStream_t s)
{
    if (r == 1) return band(seeds, coarse, band_vox, list, count, work, s);
    const BandArgs a{seeds, nvox(coarse) * r * r * r, coarse.nx * r, coarse.ny * r, band_vox * band_vox,
                     r, coarse.nx, coarse.ny};
    return band_launch<false, true>(a, ceil_div(a.N, kBandTile), nullptr, 0, list, count, work, s);
}

size_t band_batched_work_bytes(int64_t total_vox) { return band_work_points(total_vox); }

hipError_t band_batched(const BatchView& hv, const void* dplan, const int32_t* seeds, int32_t* list,
                        int32_t* count, void* work, hipStream_t s)
{
    static_assert(kBandTile == kBatchAlign, "a mask tile is one batch alignment unit");
    const BandArgs a{seeds, 0, 0, 0, 0, 1, 0, 0};
    return band_launch<true, false>(a, hv.h->total_vox / kBandTile, (const char*)dplan, hv.h->nobj, list, count,
                                    work, s);
}

hipError_t combine_batched(const BatchView& hv, const void* dplan, const int32_t* seeds, const float* dmin,
                           const uint32_t* hits, float* fine, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine_batched, dim3((unsigned)(hv.h->total_vox / kBatchAlign)), dim3(256), 0, s,
                       (const char*)dplan, hv.h->nobj, seeds, dmin, hits, fine);
    return hipGetLastError();
}

hipError_t reset_accum(float* dmin, uint32_t* hits, uint64_t* argmin, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 16384)), dim3(256),
                       0, s, dmin, hits, argmin, n);
    return hipGetLastError();
}

namespace {

template <int MODE, bool kRef>
hipError_t combine_launch(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& g, int32_t r,
                          int32_t band_vox, float beta, float bias, float alpha, int32_t first_frame,
                          int32_t consume, float* state, float* fine, hipStream_t s)
{
    dim3 grid((unsigned)ceil_div(g.nx * r, 64), (unsigned)ceil_div(g.ny * r, 4), (unsigned)(g.nz * r));
    hipLaunchKernelGGL((k_combine<MODE, kRef>), grid, dim3(256), 0, s, seeds, dmin, hits, g, r,
                       band_vox * band_vox, beta, bias, alpha, 1.0f - alpha, first_frame, consume, state, fine);
    return hipGetLastError();
}

}  // namespace

hipError_t combine_refined(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& coarse, int32_t r,
                           int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                           int32_t first_frame, int32_t consume, float* state, float* fine, hipStream_t s)
{
    if (r == 1) {
        if (mode == RTSDF_ACCUM)
            return combine_launch<RTSDF_ACCUM, false>(seeds, dmin, hits, coarse, 1, band_vox, beta, bias, alpha,
                                                      first_frame, consume, state, fine, s);
        return combine_launch<RTSDF_DECAY, false>(seeds, dmin, hits, coarse, 1, band_vox, beta, bias, alpha,
                                                  first_frame, consume, state, fine, s);
    }
    if (mode == RTSDF_ACCUM)
        return combine_launch<RTSDF_ACCUM, true>(seeds, dmin, hits, coarse, r, band_vox, beta, bias, alpha,
                                                 first_frame, consume, state, fine, s);
    return combine_launch<RTSDF_DECAY, true>(seeds, dmin, hits, coarse, r, band_vox, beta, bias, alpha,
                                             first_frame, consume, state, fine, s);
}

hipError_t combine(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& g,
                   int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                   int32_t first_frame, int32_t consume, float* state, float* fine, hipStream_t s)
{
    return combine_refined(seeds, dmin, hits, g, 1, band_vox, beta, bias, mode, alpha, first_frame, consume,
                           state, fine, s);
}

}  // namespace rtsdf
