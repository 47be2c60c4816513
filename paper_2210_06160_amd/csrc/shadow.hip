// Soft shadows by sphere tracing the fine field (section 2.4) and the reverse pass that
// carries an image gradient back to the field.
//
// One wave shades a tile of 64 pixels (8 x 8 unless tuned otherwise): neighbouring shadow rays march through
// neighbouring cells, so a wave's trilinear gathers share cache lines.  Work-groups are
// dealt to the eight XCDs round-robin; the tile order is remapped so that each XCD shades
// one contiguous band of image rows and its L2 holds the part of the field those rays cross.
// The field is read through eight scalar gathers per sample (it is 8 MiB at 128^3, so the
// gathers hit L2 / MALL, not HBM, after first touch).
//
// Reverse pass: the forward march is repeated, keeping every step's t in LDS (its sign
// bit records whether the step clamp was active), then the adjoint runs backwards from the
// minimising step and scatters into the field with binary32 atomic adds (no return value).
#include "internal.h"
#include "tuning.h"

namespace rtsdf {

namespace {

constexpr int kTX = RTSDF_SHADOW_TILE_X;  // a wave shades kTX x kTY pixels
constexpr int kTY = 64 / kTX;
static_assert(kTX * kTY == 64 && (kTX & (kTX - 1)) == 0, "a shadow tile is one wave");
constexpr int kXcds = 8;

// block b runs on XCD b % 8; XCD x receives the contiguous tile range starting at start(x)
__device__ inline int xcd_tile(int b, int nb)
{
    const int x = b % kXcds, r = b / kXcds;
    const int q = nb / kXcds, rem = nb % kXcds;
    return x * q + (x < rem ? x : rem) + r;
}

struct Axis {
    int32_t i0;     // lower corner index
    int32_t step;   // 1, or 0 on a one-point axis
    float fr;       // fraction towards the upper corner
    bool inside;    // strictly inside the box of centres (gradient is zero outside)
};

// grid coordinate c = (x - org) / h - 1/2 (centres at integers), clamped to [0, n-1]
__device__ inline Axis axis(float x, float org, float inv_h, int32_t n)
{
    Axis a;
    float c = (x - org) * inv_h - 0.5f;
    const float top = (float)(n - 1);
    a.inside = c > 0.0f && c < top;
    c = fminf(fmaxf(c, 0.0f), top);  // a NaN becomes 0
    int32_t b = (int32_t)floorf(c);
    b = b > n - 2 ? n - 2 : b;
    b = b < 0 ? 0 : b;
    a.i0 = b;
    a.step = n > 1 ? 1 : 0;
    a.fr = n > 1 ? c - (float)b : 0.0f;
    return a;
}

struct Cell {
    int64_t base;            // index of the lower corner
    int32_t sx, sy, sz;      // index strides to the upper corner per axis
    Axis ax, ay, az;
};

__device__ inline Cell cell_of(const rtsdf_grid& g, float inv_h, float3 X)
{
    Cell c;
    c.ax = axis(X.x, g.org[0], inv_h, g.nx);
    c.ay = axis(X.y, g.org[1], inv_h, g.ny);
    c.az = axis(X.z, g.org[2], inv_h, g.nz);
    c.base = c.ax.i0 + (int64_t)g.nx * (c.ay.i0 + (int64_t)g.ny * c.az.i0);
    c.sx = c.ax.step;
    c.sy = g.nx * c.ay.step;
    c.sz = g.nx * g.ny * c.az.step;
    return c;
}

// trilinear value; lerps in x, then y, then z with a + f (b - a).  If grad != nullptr it
// also returns the gradient with respect to X (zero along clamped axes).
__device__ inline float trilinear(const float* __restrict__ f, const Cell& c, float inv_h,
                                  float3* grad)
{
    const float* p = f + c.base;
    const float c000 = p[0], c001 = p[c.sx];
    const float c010 = p[c.sy], c011 = p[c.sy + c.sx];
    const float c100 = p[c.sz], c101 = p[c.sz + c.sx];
    const float c110 = p[c.sz + c.sy], c111 = p[c.sz + c.sy + c.sx];
    const float fx = c.ax.fr, fy = c.ay.fr, fz = c.az.fr;
    const float x00 = c000 + fx * (c001 - c000), x01 = c010 + fx * (c011 - c010);
    const float x10 = c100 + fx * (c101 - c100), x11 = c110 + fx * (c111 - c110);
    const float y0 = x00 + fy * (x01 - x00), y1 = x10 + fy * (x11 - x10);
    if (grad) {
        const float d00 = c001 - c000, d01 = c011 - c010, d10 = c101 - c100, d11 = c111 - c110;
        const float dy0x = d00 + fy * (d01 - d00), dy1x = d10 + fy * (d11 - d10);
        const float gx = dy0x + fz * (dy1x - dy0x);
        const float gy = (x01 - x00) + fz * ((x11 - x10) - (x01 - x00));
        const float gz = y1 - y0;
        grad->x = c.ax.inside ? gx * inv_h : 0.0f;
        grad->y = c.ay.inside ? gy * inv_h : 0.0f;
        grad->z = c.az.inside ? gz * inv_h : 0.0f;
    }
    return y0 + fz * (y1 - y0);
}

__device__ inline void scatter(float* __restrict__ gf, const Cell& c, float w)
{
    const float fx = c.ax.fr, fy = c.ay.fr, fz = c.az.fr;
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    float* p = gf + c.base;
    unsafeAtomicAdd(p, w * (gx * gy * gz));
    unsafeAtomicAdd(p + c.sx, w * (fx * gy * gz));
    unsafeAtomicAdd(p + c.sy, w * (gx * fy * gz));
    unsafeAtomicAdd(p + c.sy + c.sx, w * (fx * fy * gz));
    unsafeAtomicAdd(p + c.sz, w * (gx * gy * fz));
    unsafeAtomicAdd(p + c.sz + c.sx, w * (fx * gy * fz));
    unsafeAtomicAdd(p + c.sz + c.sy, w * (gx * fy * fz));
    unsafeAtomicAdd(p + c.sz + c.sy + c.sx, w * (fx * fy * fz));
}

__device__ inline bool pixel_of(const rtsdf_shadow& s, int tiles_x, int& a, int& b)
{
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    a = (tile % tiles_x) * kTX + (int)(threadIdx.x & (kTX - 1));
    b = (tile / tiles_x) * kTY + (int)(threadIdx.x / kTX);
    return a < s.width && b < s.height;
}

__device__ inline float3 march_point(float3 P, float t, const rtsdf_shadow& s)
{
    return make_float3(P.x + t * s.light[0], P.y + t * s.light[1], P.z + t * s.light[2]);
}

__global__ __launch_bounds__(kTX* kTY) void k_shadow_forward(const float* __restrict__ fine,
                                                                 const rtsdf_grid g, const rtsdf_shadow s,
                                                                 float inv_h, int tiles_x,
                                                                 float* __restrict__ img)
{
    int a, b;
    if (!pixel_of(s, tiles_x, a, b)) return;
    const float3 P = make_float3(s.x0 + ((float)a + 0.5f) * s.dx, s.y, s.z0 + ((float)b + 0.5f) * s.dz);
    float t = s.t0, res = 1.0f;
    for (int m = 0; m < s.steps; ++m) {
        const Cell c = cell_of(g, inv_h, march_point(P, t, s));
        const float v = trilinear(fine, c, inv_h, nullptr);
        const float r = s.k * v / t;
        res = r < res ? r : res;
        t += fminf(fmaxf(v, s.smin), s.smax);
    }
    img[(int64_t)b * s.width + a] = res > 0.0f ? res : 0.0f;
}

__global__ __launch_bounds__(kTX* kTY) void k_shadow_backward(const float* __restrict__ fine,
                                                                  const rtsdf_grid g, const rtsdf_shadow s,
                                                                  float inv_h, int tiles_x,
                                                                  const float* __restrict__ grad_img,
                                                                  float* __restrict__ grad_fine)
{
    extern __shared__ float s_t[];  // [steps][64]: t_m, negative when clamp(s_m) was active
    int a, b;
    if (!pixel_of(s, tiles_x, a, b)) return;
    const float gi = grad_img[(int64_t)b * s.width + a];
    if (gi == 0.0f) return;
    const int lane = (int)threadIdx.x;
    const float3 P = make_float3(s.x0 + ((float)a + 0.5f) * s.dx, s.y, s.z0 + ((float)b + 0.5f) * s.dz);
    float t = s.t0, res = 1.0f, s_best = 0.0f, t_best = 1.0f;
    int best = -1;
    for (int m = 0; m < s.steps; ++m) {
        const Cell c = cell_of(g, inv_h, march_point(P, t, s));
        const float v = trilinear(fine, c, inv_h, nullptr);
        const float r = s.k * v / t;
        if (r < res) {
            res = r;
            best = m;
            s_best = v;
            t_best = t;
        }
        s_t[m * (kTX * kTY) + lane] = (v > s.smin && v < s.smax) ? t : -t;
        t += fminf(fmaxf(v, s.smin), s.smax);
    }
    if (best < 0 || !(res > 0.0f)) return;
    // res = k s / t at the minimising step
    float sbar = gi * s.k / t_best;
    float tbar = -gi * s.k * s_best / (t_best * t_best);
    for (int m = best; m >= 0; --m) {
        const float tm = fabsf(s_t[m * (kTX * kTY) + lane]);
        const Cell c = cell_of(g, inv_h, march_point(P, tm, s));
        float3 gr;
        trilinear(fine, c, inv_h, &gr);
        scatter(grad_fine, c, sbar);
        tbar += sbar * ((gr.x * s.light[0] + gr.y * s.light[1]) + gr.z * s.light[2]);
        if (m == 0) break;
        // t_m = t_{m-1} + clamp(s_{m-1}): s_{m-1} receives tbar where the clamp is inactive
        sbar = s_t[(m - 1) * (kTX * kTY) + lane] > 0.0f ? tbar : 0.0f;
    }
}

int tiles(int n, int t) { return (n + t - 1) / t; }

}  // namespace

hipError_t shadow_forward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s, float* img,
                          hipStream_t st)
{
    if (s.width == 0 || s.height == 0) return hipSuccess;
    const int tx = tiles(s.width, kTX), nb = tx * tiles(s.height, kTY);
    k_shadow_forward<<<nb, kTX * kTY, 0, st>>>(fine, g, s, 1.0f / g.h, tx, img);
    return hipGetLastError();
}

hipError_t shadow_backward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s,
                           const float* grad_img, float* grad_fine, hipStream_t st)
{
    if (s.width == 0 || s.height == 0) return hipSuccess;
    const int tx = tiles(s.width, kTX), nb = tx * tiles(s.height, kTY);
    const size_t lds = sizeof(float) * (size_t)s.steps * kTX * kTY;
    k_shadow_backward<<<nb, kTX * kTY, lds, st>>>(fine, g, s, 1.0f / g.h, tx, grad_img, grad_fine);
    return hipGetLastError();
}

}  // namespace rtsdf
