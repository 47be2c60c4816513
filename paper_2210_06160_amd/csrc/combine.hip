// Ray mask compaction (section 2.3), accumulator reset, and the coarse/fine combination
// (section 2.1 running minimum, section 2.5.1 Eq. 1 decay, section 2.5.3 bias).
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kBandThreads = 256;
constexpr int kBandItems = 16;  // consecutive voxels per thread
constexpr int kBandTile = kBandThreads * kBandItems;

__device__ inline int32_t seed_d2(int32_t s, int32_t x, int32_t y, int32_t z)
{
    const int32_t dx = (s & 1023) - x, dy = ((s >> 10) & 1023) - y, dz = ((s >> 20) & 1023) - z;
    return dx * dx + dy * dy + dz * dz;
}

// Flags of the kBandItems voxels of this thread, as a bit mask.
__device__ uint32_t band_bits(const int32_t* __restrict__ seeds, int64_t N, int32_t nx, int32_t ny,
                              int32_t b2, int64_t first)
{
    uint32_t bits = 0;
    if (first >= N) return 0;
    int64_t row = first / nx;
    int32_t x = (int32_t)(first - row * nx);
    int32_t y = (int32_t)(row % ny);
    int32_t z = (int32_t)(row / ny);
#pragma unroll
    for (int i = 0; i < kBandItems; ++i) {
        const int64_t p = first + i;
        if (p < N) {
            const int32_t s = seeds[p];
            if (s != RTSDF_EMPTY && seed_d2(s, x, y, z) <= b2) bits |= 1u << i;
        }
        if (++x == nx) {
            x = 0;
            if (++y == ny) {
                y = 0;
                ++z;
            }
        }
    }
    return bits;
}

// The grid a mask work-group scans.  Single object: the arguments.  Batch: the object that
// owns the work-group's tile (tiles are kBatchAlign = kBandTile voxels and never straddle
// objects); `base` is added to the listed indices.
struct BandGrid {
    const int32_t* seeds;
    int64_t N, first, base;
    int32_t nx, ny, b2;
};

template <bool kBatch>
__device__ inline BandGrid band_grid(const int32_t* seeds, int64_t N, int32_t nx, int32_t ny, int32_t b2,
                                     const char* plan, int32_t nobj)
{
    const int64_t tile = (int64_t)blockIdx.x * kBandTile;
    if (!kBatch) return BandGrid{seeds, N, tile + (int64_t)threadIdx.x * kBandItems, 0, nx, ny, b2};
    const BatchView v = batch_view(plan, nobj);
    const BatchObject& ob = v.obj[find_object(v.vox_prefix, nobj, tile)];
    return BandGrid{seeds + ob.vox_off, nvox(ob.g), tile - ob.vox_off + (int64_t)threadIdx.x * kBandItems,
                    ob.vox_off, ob.g.nx, ob.g.ny, ob.band_vox * ob.band_vox};
}

template <bool kBatch>
__global__ __launch_bounds__(kBandThreads) void k_band_count(const int32_t* __restrict__ seeds,
                                                             int64_t N, int32_t nx, int32_t ny,
                                                             int32_t b2, uint32_t* __restrict__ counts,
                                                             const char* plan, int32_t nobj)
{
    __shared__ uint32_t part[kBandThreads / kWave];
    const BandGrid bg = band_grid<kBatch>(seeds, N, nx, ny, b2, plan, nobj);
    uint32_t c = __popc(band_bits(bg.seeds, bg.N, bg.nx, bg.ny, bg.b2, bg.first));
    for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBandThreads / kWave; ++w) t += part[w];
        counts[blockIdx.x] = t;
    }
}

template <bool kBatch>
__global__ __launch_bounds__(kBandThreads) void k_band_write(const int32_t* __restrict__ seeds,
                                                             int64_t N, int32_t nx, int32_t ny,
                                                             int32_t b2,
                                                             const uint32_t* __restrict__ offsets,
                                                             int32_t* __restrict__ list, const char* plan,
                                                             int32_t nobj)
{
    __shared__ uint32_t part[kBandThreads / kWave];
    const BandGrid bg = band_grid<kBatch>(seeds, N, nx, ny, b2, plan, nobj);
    const uint32_t bits = band_bits(bg.seeds, bg.N, bg.nx, bg.ny, bg.b2, bg.first);
    const uint32_t c = __popc(bits);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t inc = c;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) part[wave] = inc;
    __syncthreads();
    uint32_t pos = offsets[blockIdx.x] + inc - c;
    for (int w = 0; w < wave; ++w) pos += part[w];
    for (int i = 0; i < kBandItems; ++i)
        if (bits & (1u << i)) list[pos++] = (int32_t)(bg.base + bg.first + i);
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

template <int MODE>
__global__ __launch_bounds__(256) void k_combine(const int32_t* __restrict__ seeds,
                                                 float* __restrict__ dmin,
                                                 uint32_t* __restrict__ hits, const rtsdf_grid g,
                                                 int32_t b2, float beta, float bias, float alpha,
                                                 float one_minus_alpha, int32_t first_frame,
                                                 int32_t consume, float* __restrict__ state,
                                                 float* __restrict__ fine)
{
    const int32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int32_t y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int32_t z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int64_t p = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
    const int32_t s = seeds[p];
    float u = __int_as_float(0x7f800000);
    bool inband = false;
    if (s != RTSDF_EMPTY) {
        const int32_t d2 = seed_d2(s, x, y, z);
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

size_t band_work_bytes(const rtsdf_grid& g)
{
    const int64_t nb = ceil_div(nvox(g), kBandTile);
    return align256((size_t)nb * 4) + align256(4) + scan_work_bytes_u32(nb);
}

hipError_t band(const int32_t* seeds, const rtsdf_grid& g, int32_t band_vox, int32_t* list,
                int32_t* count, void* work, hipStream_t s)
{
    const int64_t N = nvox(g);
    const int64_t nb = ceil_div(N, kBandTile);
    char* w = (char*)work;
    uint32_t* counts = (uint32_t*)w;
    w += align256((size_t)nb * 4);
    uint32_t* total = (uint32_t*)w;
    w += align256(4);
    const int32_t b2 = band_vox * band_vox;
    hipLaunchKernelGGL(k_band_count<false>, dim3((unsigned)nb), dim3(kBandThreads), 0, s, seeds, N, g.nx,
                       g.ny, b2, counts, nullptr, 0);
    hipError_t e = scan_exclusive_u32(counts, counts, nb, total, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_write<false>, dim3((unsigned)nb), dim3(kBandThreads), 0, s, seeds, N, g.nx,
                       g.ny, b2, (const uint32_t*)counts, list, nullptr, 0);
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, (const uint32_t*)total, count);
    return hipGetLastError();
}

size_t band_batched_work_bytes(int64_t total_vox)
{
    const int64_t nb = ceil_div(total_vox, kBandTile);
    return align256((size_t)nb * 4) + align256(4) + scan_work_bytes_u32(nb);
}

hipError_t band_batched(const BatchView& hv, const void* dplan, const int32_t* seeds, int32_t* list,
                        int32_t* count, void* work, hipStream_t s)
{
    static_assert(kBandTile == kBatchAlign, "a mask tile is one batch alignment unit");
    const int64_t nb = hv.h->total_vox / kBandTile;
    const char* plan = (const char*)dplan;
    const int32_t nobj = hv.h->nobj;
    char* w = (char*)work;
    uint32_t* counts = (uint32_t*)w;
    w += align256((size_t)nb * 4);
    uint32_t* total = (uint32_t*)w;
    w += align256(4);
    hipLaunchKernelGGL(k_band_count<true>, dim3((unsigned)nb), dim3(kBandThreads), 0, s, seeds, (int64_t)0, 0, 0,
                       0, counts, plan, nobj);
    hipError_t e = scan_exclusive_u32(counts, counts, nb, total, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_write<true>, dim3((unsigned)nb), dim3(kBandThreads), 0, s, seeds, (int64_t)0, 0, 0,
                       0, (const uint32_t*)counts, list, plan, nobj);
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, (const uint32_t*)total, count);
    return hipGetLastError();
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

hipError_t combine(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& g,
                   int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                   int32_t first_frame, int32_t consume, float* state, float* fine, hipStream_t s)
{
    dim3 grid((unsigned)ceil_div(g.nx, 64), (unsigned)ceil_div(g.ny, 4), (unsigned)g.nz);
    const float oma = 1.0f - alpha;
    const int32_t b2 = band_vox * band_vox;
    if (mode == RTSDF_ACCUM)
        hipLaunchKernelGGL(k_combine<RTSDF_ACCUM>, grid, dim3(256), 0, s, seeds, dmin, hits, g, b2,
                           beta, bias, alpha, oma, first_frame, consume, state, fine);
    else
        hipLaunchKernelGGL(k_combine<RTSDF_DECAY>, grid, dim3(256), 0, s, seeds, dmin, hits, g, b2,
                           beta, bias, alpha, oma, first_frame, consume, state, fine);
    return hipGetLastError();
}

}  // namespace rtsdf
