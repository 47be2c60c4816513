// One jump-flooding pass (section 2.2) over packed int32 seed ids.
//
// Query order: the stored seed first (rank 0), then the 26 offsets e in {-1,0,1}^3 \ {0}
// in the order ez, ey, ex ascending (ranks 1..26).  A later query replaces the incumbent
// only when strictly closer, which is the same as taking the minimum of the 32-bit key
// (d2 << 5) | rank: d2 < 2^22 for grids up to 1024^3, so the key never overflows and
// the reduction is order-free (v_min3_u32 on gfx950).
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kBX = 64, kBY = 4;

__device__ inline uint32_t sq_dist(int32_t s, int32_t x, int32_t y, int32_t z)
{
    const int32_t dx = (s & 1023) - x;
    const int32_t dy = ((s >> 10) & 1023) - y;
    const int32_t dz = ((s >> 20) & 1023) - z;
    return (uint32_t)(dx * dx + dy * dy + dz * dz);
}

__global__ __launch_bounds__(kBX * kBY) void k_jfa_direct(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int32_t nx,
                                                          int32_t ny, int32_t nz, int32_t k)
{
    const int32_t x = blockIdx.x * kBX + threadIdx.x;
    const int32_t y = blockIdx.y * kBY + threadIdx.y;
    const int32_t z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t p = x + (int64_t)nx * y + plane * z;
    uint32_t best = 0xFFFFFFFFu;
    int32_t bid = RTSDF_EMPTY;
    {
        const int32_t s = in[p];
        if (s != RTSDF_EMPTY) {
            best = sq_dist(s, x, y, z) << 5;
            bid = s;
        }
    }
    uint32_t rank = 0;
#pragma unroll
    for (int ez = -1; ez <= 1; ++ez) {
#pragma unroll
        for (int ey = -1; ey <= 1; ++ey) {
#pragma unroll
            for (int ex = -1; ex <= 1; ++ex) {
                if (ex == 0 && ey == 0 && ez == 0) continue;
                ++rank;
                const int32_t qx = x + ex * k, qy = y + ey * k, qz = z + ez * k;
                if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) continue;
                const int32_t s = in[qx + (int64_t)nx * qy + plane * qz];
                if (s == RTSDF_EMPTY) continue;
                const uint32_t key = (sq_dist(s, x, y, z) << 5) | rank;
                if (key < best) {
                    best = key;
                    bid = s;
                }
            }
        }
    }
    out[p] = bid;
}

}  // namespace

hipError_t jfa_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, hipStream_t s)
{
    dim3 grid((unsigned)ceil_div(g.nx, kBX), (unsigned)ceil_div(g.ny, kBY), (unsigned)g.nz);
    hipLaunchKernelGGL(k_jfa_direct, grid, dim3(kBX, kBY), 0, s, in, out, g.nx, g.ny, g.nz, k);
    return hipGetLastError();
}

}  // namespace rtsdf
