// Soft shadows by sphere tracing the fine field (section 2.4) and the reverse pass that
// carries an image gradient back to the field.  One launch shades every light's image
// (blockIdx.y is the light); the start offset may be jittered along the light per pixel,
// light and frame, and the closest-approach estimate may be triangulated from two
// consecutive samples (section 2.5.2).
//
// One wave shades a tile of 64 pixels (RTSDF_SHADOW_TILE_X wide: 4 x 16 as tuned):
// neighbouring shadow rays march through neighbouring cells, so a wave's trilinear gathers
// share cache lines.  Work-groups are
// dealt to the eight XCDs round-robin; the tile order is remapped so that each XCD shades
// one contiguous band of image rows and its L2 holds the part of the field those rays cross.
// The field is read through eight scalar gathers per sample (it is 8 MiB at 128^3, so the
// gathers hit L2 / MALL, not HBM, after first touch).
//
// Reverse pass: the forward march is repeated, keeping every step's t in LDS (its sign
// bit records whether the step clamp was active), then the adjoint runs backwards from the
// minimising step and scatters into the field with binary32 atomic adds (no return value).
#include "internal.h"
#include "sampling.h"
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
    float inv_h;             // 1 / h of the grid the cell belongs to
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
    c.inv_h = inv_h;
    return c;
}

// trilinear value; lerps in x, then y, then z with a + f (b - a).  If grad != nullptr it
// also returns the gradient with respect to X (zero along clamped axes).
__device__ inline float trilinear(const float* __restrict__ f, const Cell& c, float3* grad)
{
    const float inv_h = c.inv_h;
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

// Adds w times the trilinear weights of sample cell c to its eight corners of gf.  The lanes
// of a wave often sample the same cell (neighbouring pixels march side by side, several per
// voxel) and device-scope atomics serialise at the memory side, so the active lanes are
// grouped by cell (lower corner and clamped axes), members add their eight corner values
// into their group leader's LDS slots, and each leader issues the eight atomics once.
// acc: [8][64] LDS; the block is one wave.
__device__ inline void scatter_wave(float* __restrict__ gf, const Cell& c, float w, float (*acc)[64])
{
    const int lane = (int)threadIdx.x;
    const float fx = c.ax.fr, fy = c.ay.fr, fz = c.az.fr;
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    const float v[8] = {w * (gx * gy * gz), w * (fx * gy * gz), w * (gx * fy * gz), w * (fx * fy * gz),
                        w * (gx * gy * fz), w * (fx * gy * fz), w * (gx * fy * fz), w * (fx * fy * fz)};
    const int64_t key = c.base * 8 + (c.sx != 0 ? 1 : 0) + (c.sy != 0 ? 2 : 0) + (c.sz != 0 ? 4 : 0);
    int leader = lane;
    uint64_t pending = __ballot(1);  // the lanes taking part
    while (pending != 0ull) {
        const int l = __ffsll((long long)pending) - 1;
        const int64_t kl = __shfl(key, l);
        const bool mine = key == kl;
        if (mine) leader = l;
        pending &= ~__ballot(mine);
    }
    // LDS operations of one wave complete in order; the waits make that explicit
    if (leader == lane)
        for (int i = 0; i < 8; ++i) acc[i][lane] = 0.0f;
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < 8; ++i) atomicAdd(&acc[i][leader], v[i]);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    if (leader == lane) {
        float* p = gf + c.base;
        unsafeAtomicAdd(p, acc[0][lane]);
        unsafeAtomicAdd(p + c.sx, acc[1][lane]);
        unsafeAtomicAdd(p + c.sy, acc[2][lane]);
        unsafeAtomicAdd(p + c.sy + c.sx, acc[3][lane]);
        unsafeAtomicAdd(p + c.sz, acc[4][lane]);
        unsafeAtomicAdd(p + c.sz + c.sx, acc[5][lane]);
        unsafeAtomicAdd(p + c.sz + c.sy, acc[6][lane]);
        unsafeAtomicAdd(p + c.sz + c.sy + c.sx, acc[7][lane]);
    }
}

// Everything a launch needs besides the field: the receiver lattice and march constants,
// the lights, and the jitter draw.
struct March {
    rtsdf_shadow s;                     // s.light is not used
    float light[RTSDF_MAX_LIGHTS][3];
    float jitter;                       // start offset t0 + jitter * u
    uint32_t frame, k0, k1;             // counter word and key of the jitter draw
    int32_t bounded;                    // end the march where it leaves the grid's box
};

// whether X lies in the grid's box [org, org + n h] (closed)
__device__ inline bool in_box(const rtsdf_grid& g, float inv_h, float3 X)
{
    const float cx = (X.x - g.org[0]) * inv_h, cy = (X.y - g.org[1]) * inv_h, cz = (X.z - g.org[2]) * inv_h;
    return cx >= 0.0f && cx <= (float)g.nx && cy >= 0.0f && cy <= (float)g.ny && cz >= 0.0f && cz <= (float)g.nz;
}

// The field a march samples.  GridField: one grid.  ClipField: the levels of a clip map,
// finest first, concatenated at voxel offsets off[l]; a point reads the finest level whose
// box of grid-point centres holds it (grid coordinate (X - org)/h - 1/2 in [0, n-1] on every
// axis), the coarsest (clamped) when none does; a bounded march ends at the coarsest box.
struct GridField {
    rtsdf_grid g;
    float inv_h;
    __device__ Cell cell(float3 X, int* level = nullptr) const
    {
        if (level) *level = 0;
        return cell_of(g, inv_h, X);
    }
    __device__ bool in_bounds(float3 X) const { return in_box(g, inv_h, X); }
};

struct ClipField {
    int32_t L;
    rtsdf_grid g[RTSDF_MAX_CLIP_LEVELS];
    float inv_h[RTSDF_MAX_CLIP_LEVELS];
    int64_t off[RTSDF_MAX_CLIP_LEVELS];
    __device__ Cell cell(float3 X, int* level = nullptr) const
    {
        int l = 0;
        for (; l < L - 1; ++l) {
            const rtsdf_grid& q = g[l];
            const float cx = (X.x - q.org[0]) * inv_h[l] - 0.5f, cy = (X.y - q.org[1]) * inv_h[l] - 0.5f,
                        cz = (X.z - q.org[2]) * inv_h[l] - 0.5f;
            if (cx >= 0.0f && cx <= (float)(q.nx - 1) && cy >= 0.0f && cy <= (float)(q.ny - 1) && cz >= 0.0f &&
                cz <= (float)(q.nz - 1))
                break;
        }
        if (level) *level = l;
        Cell c = cell_of(g[l], inv_h[l], X);
        c.base += off[l];
        return c;
    }
    __device__ bool in_bounds(float3 X) const { return in_box(g[L - 1], inv_h[L - 1], X); }
};

__device__ inline float clamp_step(const rtsdf_shadow& s, float v) { return fminf(fmaxf(v, s.smin), s.smax); }

// Two-sample estimate of the closest approach: samples r1 and r2 one clamped step delta
// apart bound empty spheres; their intersection circle lies y behind the later sample with
// radius d, giving k d / (t - y); without a circle (or behind the start) the one-sample
// k r2 / t.  Returns the estimate and whether the circle was used.
__device__ inline float triangulate(float r1, float r2, float delta, float t, float k, bool& valid)
{
    const float y = (r2 * r2 - r1 * r1 + delta * delta) / (2.0f * delta);
    const float d2 = r2 * r2 - y * y;
    valid = r1 > 0.0f && r2 > 0.0f && d2 > 0.0f && t - y > 0.0f;
    return valid ? k * sqrtf(d2) / (t - y) : k * r2 / t;
}

__device__ inline float start_offset(const March& M, int64_t pixel, int light)
{
    if (M.jitter == 0.0f) return M.s.t0;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)pixel, M.frame, (uint32_t)light, 0xFFFFFFFFu), M.k0, M.k1);
    const float u = (float)(w.x >> 8) * (1.0f / 16777216.0f);
    return M.s.t0 + M.jitter * u;
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

template <bool kTri, class Field>
__global__ __launch_bounds__(kTX* kTY) void k_shadow_forward(const float* __restrict__ fine, const Field F,
                                                                 const March M, int tiles_x,
                                                                 float* __restrict__ img)
{
    const rtsdf_shadow& s = M.s;
    int a, b;
    if (!pixel_of(s, tiles_x, a, b)) return;
    const int l = (int)blockIdx.y;
    const float3 L = make_float3(M.light[l][0], M.light[l][1], M.light[l][2]);
    const int64_t pix = (int64_t)b * s.width + a;
    const float3 P = make_float3(s.x0 + ((float)a + 0.5f) * s.dx, s.y, s.z0 + ((float)b + 0.5f) * s.dz);
    float t = start_offset(M, pix, l), res = 1.0f, prev = 0.0f;
    for (int m = 0; m < s.steps; ++m) {
        const float3 X = make_float3(P.x + t * L.x, P.y + t * L.y, P.z + t * L.z);
        if (M.bounded && !F.in_bounds(X)) break;
        const Cell c = F.cell(X);
        const float v = trilinear(fine, c, nullptr);
        float r;
        if (kTri && m > 0) {
            bool valid;
            r = triangulate(prev, v, clamp_step(s, prev), t, s.k, valid);
        } else {
            r = s.k * v / t;
        }
        res = r < res ? r : res;
        prev = v;
        t += clamp_step(s, v);
    }
    img[(int64_t)l * s.width * s.height + pix] = res > 0.0f ? res : 0.0f;
}

template <bool kTri, class Field>
__global__ __launch_bounds__(kTX* kTY) void k_shadow_backward(const float* __restrict__ fine, const Field F,
                                                                  const March M, int tiles_x,
                                                                  const float* __restrict__ grad_img,
                                                                  float* __restrict__ grad_fine)
{
    extern __shared__ float s_t[];  // [steps][64]: t_m, negative when clamp(s_m) was active
    __shared__ float s_acc[8][64];  // scatter_wave's group sums
    const rtsdf_shadow& s = M.s;
    int a, b;
    if (!pixel_of(s, tiles_x, a, b)) return;
    const int l = (int)blockIdx.y;
    const int64_t pix = (int64_t)b * s.width + a;
    const float gi = grad_img[(int64_t)l * s.width * s.height + pix];
    if (gi == 0.0f) return;
    const float3 L = make_float3(M.light[l][0], M.light[l][1], M.light[l][2]);
    const int lane = (int)threadIdx.x;
    const float3 P = make_float3(s.x0 + ((float)a + 0.5f) * s.dx, s.y, s.z0 + ((float)b + 0.5f) * s.dz);
    float t = start_offset(M, pix, l), res = 1.0f, prev = 0.0f;
    float s_best = 0.0f, s_prev_best = 0.0f, t_best = 1.0f;
    bool tri_best = false;
    int best = -1;
    for (int m = 0; m < s.steps; ++m) {
        const float3 X = make_float3(P.x + t * L.x, P.y + t * L.y, P.z + t * L.z);
        if (M.bounded && !F.in_bounds(X)) break;
        const Cell c = F.cell(X);
        const float v = trilinear(fine, c, nullptr);
        float r;
        bool valid = false;
        if (kTri && m > 0)
            r = triangulate(prev, v, clamp_step(s, prev), t, s.k, valid);
        else
            r = s.k * v / t;
        if (r < res) {
            res = r;
            best = m;
            s_best = v;
            s_prev_best = prev;
            t_best = t;
            tri_best = valid;
        }
        s_t[m * (kTX * kTY) + lane] = (v > s.smin && v < s.smax) ? t : -t;
        prev = v;
        t += clamp_step(s, v);
    }
    if (best < 0 || !(res > 0.0f)) return;
    float sbar, tbar, extra = 0.0f;  // extra: direct adjoint of s_{best-1}
    if (kTri && tri_best) {
        // res = k D / (T - y), D = sqrt(r2^2 - y^2), y = (r2^2 - r1^2 + delta^2) / (2 delta)
        const float r1 = s_prev_best, r2 = s_best, T = t_best, delta = clamp_step(s, r1);
        const float y = (r2 * r2 - r1 * r1 + delta * delta) / (2.0f * delta);
        const float D = sqrtf(r2 * r2 - y * y);
        const float dy_r2 = r2 / delta, dy_r1 = -r1 / delta, dy_dl = 1.0f - y / delta;
        const float dD_r2 = (r2 - y * dy_r2) / D, dD_r1 = -y * dy_r1 / D, dD_dl = -y * dy_dl / D;
        const float ka = s.k / (T - y), kc = res / (T - y);
        sbar = gi * (ka * dD_r2 + kc * dy_r2);
        tbar = -gi * kc;
        extra = gi * (ka * dD_r1 + kc * dy_r1);
        if (r1 > s.smin && r1 < s.smax) extra += gi * (ka * dD_dl + kc * dy_dl);
    } else {
        sbar = gi * s.k / t_best;
        tbar = -gi * s.k * s_best / (t_best * t_best);
    }
    for (int m = best; m >= 0; --m) {
        const float tm = fabsf(s_t[m * (kTX * kTY) + lane]);
        const Cell c = F.cell(make_float3(P.x + tm * L.x, P.y + tm * L.y, P.z + tm * L.z));
        float3 gr;
        trilinear(fine, c, &gr);
        scatter_wave(grad_fine, c, sbar, s_acc);
        tbar += sbar * ((gr.x * L.x + gr.y * L.y) + gr.z * L.z);
        if (m == 0) break;
        // t_m = t_{m-1} + clamp(s_{m-1}): s_{m-1} receives tbar where the clamp is inactive
        sbar = s_t[(m - 1) * (kTX * kTY) + lane] > 0.0f ? tbar : 0.0f;
        if (kTri && m == best) sbar += extra;
    }
}

int tiles(int n, int t) { return (n + t - 1) / t; }

March make_march(const rtsdf_shadow& s, const float (*lights)[3], int32_t nlights, float jitter, uint32_t frame,
                 uint64_t key, int32_t bounded)
{
    March M;
    M.bounded = bounded;
    M.s = s;
    for (int l = 0; l < RTSDF_MAX_LIGHTS; ++l)
        for (int a = 0; a < 3; ++a) M.light[l][a] = l < nlights ? lights[l][a] : 0.0f;
    M.jitter = jitter;
    M.frame = frame;
    M.k0 = (uint32_t)key;
    M.k1 = (uint32_t)(key >> 32);
    return M;
}

template <class Field>
hipError_t forward(const float* fine, const Field& F, const March& M, int32_t nlights, bool tri, float* img,
                   hipStream_t st)
{
    const rtsdf_shadow& s = M.s;
    if (s.width == 0 || s.height == 0) return hipSuccess;
    const int tx = tiles(s.width, kTX);
    const dim3 grid((unsigned)(tx * tiles(s.height, kTY)), (unsigned)nlights);
    if (tri)
        k_shadow_forward<true, Field><<<grid, kTX * kTY, 0, st>>>(fine, F, M, tx, img);
    else
        k_shadow_forward<false, Field><<<grid, kTX * kTY, 0, st>>>(fine, F, M, tx, img);
    return hipGetLastError();
}

template <class Field>
hipError_t backward(const float* fine, const Field& F, const March& M, int32_t nlights, bool tri,
                    const float* grad_img, float* grad_fine, hipStream_t st)
{
    const rtsdf_shadow& s = M.s;
    if (s.width == 0 || s.height == 0) return hipSuccess;
    const int tx = tiles(s.width, kTX);
    const dim3 grid((unsigned)(tx * tiles(s.height, kTY)), (unsigned)nlights);
    const size_t lds = sizeof(float) * (size_t)s.steps * kTX * kTY;
    if (tri)
        k_shadow_backward<true, Field><<<grid, kTX * kTY, lds, st>>>(fine, F, M, tx, grad_img, grad_fine);
    else
        k_shadow_backward<false, Field><<<grid, kTX * kTY, lds, st>>>(fine, F, M, tx, grad_img, grad_fine);
    return hipGetLastError();
}

GridField grid_field(const rtsdf_grid& g) { return GridField{g, 1.0f / g.h}; }

ClipField clip_field(const BatchView& hv)
{
    ClipField F;
    F.L = hv.h->nobj;
    for (int l = 0; l < RTSDF_MAX_CLIP_LEVELS; ++l) {
        const int q = l < F.L ? l : F.L - 1;
        F.g[l] = hv.obj[q].g;
        F.inv_h[l] = 1.0f / hv.obj[q].g.h;
        F.off[l] = hv.obj[q].vox_off;
    }
    return F;
}

// one thread per point: the value (and level) a clip map gives it
__global__ __launch_bounds__(256) void k_clip_sample(const float* __restrict__ fine, const ClipField F,
                                                     const float* __restrict__ pts, int64_t n,
                                                     float* __restrict__ vals, int32_t* __restrict__ levels)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int l;
    const Cell c = F.cell(make_float3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]), &l);
    vals[i] = trilinear(fine, c, nullptr);
    if (levels) levels[i] = l;
}

}  // namespace

hipError_t shadow_forward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s, float* img,
                          hipStream_t st)
{
    return forward(fine, grid_field(g), make_march(s, &s.light, 1, 0.0f, 0, 0, 0), 1, false, img, st);
}

hipError_t shadow_backward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s,
                           const float* grad_img, float* grad_fine, hipStream_t st)
{
    return backward(fine, grid_field(g), make_march(s, &s.light, 1, 0.0f, 0, 0, 0), 1, false, grad_img, grad_fine,
                    st);
}

hipError_t shadow_forward_ex(const float* fine, const rtsdf_grid& g, const rtsdf_shadow_ex& s, float* img,
                             hipStream_t st)
{
    return forward(fine, grid_field(g), make_march(s.base, s.lights, s.nlights, s.jitter, s.frame, s.key, s.bounded != 0),
                   s.nlights, s.triangulate != 0, img, st);
}

hipError_t shadow_backward_ex(const float* fine, const rtsdf_grid& g, const rtsdf_shadow_ex& s,
                              const float* grad_img, float* grad_fine, hipStream_t st)
{
    return backward(fine, grid_field(g), make_march(s.base, s.lights, s.nlights, s.jitter, s.frame, s.key, s.bounded != 0),
                    s.nlights, s.triangulate != 0, grad_img, grad_fine, st);
}

hipError_t shadow_forward_clip(const BatchView& hv, const float* fine, const rtsdf_shadow_ex& s, float* img,
                               hipStream_t st)
{
    return forward(fine, clip_field(hv), make_march(s.base, s.lights, s.nlights, s.jitter, s.frame, s.key, s.bounded != 0),
                   s.nlights, s.triangulate != 0, img, st);
}

hipError_t shadow_backward_clip(const BatchView& hv, const float* fine, const rtsdf_shadow_ex& s,
                                const float* grad_img, float* grad_fine, hipStream_t st)
{
    return backward(fine, clip_field(hv), make_march(s.base, s.lights, s.nlights, s.jitter, s.frame, s.key, s.bounded != 0),
                    s.nlights, s.triangulate != 0, grad_img, grad_fine, st);
}

hipError_t clip_sample(const BatchView& hv, const float* fine, const float* pts, int64_t n, float* vals,
                       int32_t* levels, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clip_sample, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, fine, clip_field(hv), pts, n,
                       vals, levels);
    return hipGetLastError();
}

}  // namespace rtsdf
