// Device helpers for ray sampling (section 2.1): counter-based random directions and the
// binary32 ray/triangle hit.  The operation order is part of the definition (it decides
// hit/miss and front/back exactly), so the library is built with -ffp-contract=off and
// these functions must not be rewritten with fused or reassociated arithmetic.
#pragma once

#include "internal.h"

namespace rtsdf {

// Philox4x32 with 10 rounds (Salmon et al., SC 2011): multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product in one multiply-add instead of separate low and
        // high multiplies
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform direction on the unit sphere by Marsaglia's (1972) method.  Counter words:
// (voxel, frame, ray, object << 8 | attempt); each Philox call offers two (v1, v2) pairs.
__device__ inline float3 sphere_direction(uint32_t k0, uint32_t k1, uint32_t vid, uint32_t frame,
                                          uint32_t ray, uint32_t obj)
{
    for (uint32_t att = 0; att < 256u; ++att) {
        const uint4 r = philox4x32_10(make_uint4(vid, frame, ray, (obj << 8) | att), k0, k1);
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            const float a = 2.0f * ((float)(w[2 * pr] >> 8) * 0x1p-24f) - 1.0f;
            const float b = 2.0f * ((float)(w[2 * pr + 1] >> 8) * 0x1p-24f) - 1.0f;
            const float s = a * a + b * b;
            if (s < 1.0f) {
                const float q = sqrtf(1.0f - s);
                return make_float3((2.0f * a) * q, (2.0f * b) * q, 1.0f - 2.0f * s);
            }
        }
    }
    return make_float3(0.0f, 0.0f, 1.0f);
}

__device__ inline float dot3(float3 a, float3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ inline float3 cross3(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Least and greatest of three finite values.  fminf / fmaxf may return either zero when
// given -0 and +0; the box test below cannot tell the two apart (x - pad and x + pad are
// the same for both zeros when pad != 0, and comparisons treat them as equal), so its
// decisions are those of any other exact min / max.
__device__ inline float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ inline float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// Moller-Trumbore (1997).  Returns t > 0 on a hit (and sets front = det > 0, i.e. the ray
// meets the outward face), or a negative value on a miss.  A hit also needs the computed
// point o + t*w inside the triangle's box widened by `pad` on every side.
__device__ inline float hit_triangle(float3 o, float3 w, float3 v0, float3 v1, float3 v2, float pad,
                                     bool& front)
{
    const float3 e1 = make_float3(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z);
    const float3 e2 = make_float3(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z);
    const float3 P = cross3(w, e2);
    const float det = dot3(e1, P);
    if (det == 0.0f) return -1.0f;
    const float inv = 1.0f / det;
    const float3 T = make_float3(o.x - v0.x, o.y - v0.y, o.z - v0.z);
    const float u = dot3(T, P) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) return -1.0f;
    const float3 Q = cross3(T, e1);
    const float v = dot3(w, Q) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) return -1.0f;
    const float t = dot3(e2, Q) * inv;
    if (!(t > 0.0f)) return -1.0f;
    const float qx = o.x + t * w.x, qy = o.y + t * w.y, qz = o.z + t * w.z;
    // all six bounds evaluated (no short circuit): one straight-line test per wave
    const bool in_x = (qx >= min3f(v0.x, v1.x, v2.x) - pad) & (qx <= max3f(v0.x, v1.x, v2.x) + pad);
    const bool in_y = (qy >= min3f(v0.y, v1.y, v2.y) - pad) & (qy <= max3f(v0.y, v1.y, v2.y) + pad);
    const bool in_z = (qz >= min3f(v0.z, v1.z, v2.z) - pad) & (qz <= max3f(v0.z, v1.z, v2.z) + pad);
    if (!(in_x & in_y & in_z)) return -1.0f;
    front = det > 0.0f;
    return t;
}

__device__ inline float3 voxel_centre(const rtsdf_grid& g, int64_t vid, uint32_t& i, uint32_t& j,
                                      uint32_t& k)
{
    const int64_t row = vid / g.nx;
    i = (uint32_t)(vid - row * g.nx);
    j = (uint32_t)(row % g.ny);
    k = (uint32_t)(row / g.ny);
    return make_float3(g.org[0] + g.h * ((float)i + 0.5f), g.org[1] + g.h * ((float)j + 0.5f),
                       g.org[2] + g.h * ((float)k + 0.5f));
}

}  // namespace rtsdf
