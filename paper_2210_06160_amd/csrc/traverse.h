// Helpers shared by the kernels that trace rays through the 4-wide hierarchy written by
// lbvh.hip: the slab test of a child box, the sort key of a child, and bounds of the
// per-lane traversal stack.  Box tests may round freely: every triangle box is widened by
// 2*pad while a hit's computed point must lie within pad of its triangle's box, so a box
// holding a hit is never culled and traversal returns the brute-force least (t, index).
#pragma once

#include "sampling.h"

namespace rtsdf {

constexpr int kMaxStack = 176;  // <= 3 pushes per level + 1; tree depth <= 56
constexpr int32_t kNone = 0x7FFFFFFF;
constexpr uint32_t kMiss = 0xFFFFFFFFu;

__device__ inline float box_entry(float lx, float ly, float lz, float hx, float hy, float hz, float3 inv,
                                  float3 oinv, float tbest)
{
    const float x0 = fmaf(lx, inv.x, -oinv.x), x1 = fmaf(hx, inv.x, -oinv.x);
    const float y0 = fmaf(ly, inv.y, -oinv.y), y1 = fmaf(hy, inv.y, -oinv.y);
    const float z0 = fmaf(lz, inv.z, -oinv.z), z1 = fmaf(hz, inv.z, -oinv.z);
    const float tmin = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tbest));
    return tmin <= tmax ? tmin : __int_as_float(0x7f800000);
}

// The same test with each axis's near and far planes fetched by the ray's direction signs
// (near = lo where the reciprocal is positive, else hi): the slab intervals and so the
// result equal box_entry's, without ordering each axis's two planes.
__device__ inline float box_entry_nf(float nx, float ny, float nz, float fx, float fy, float fz, float3 inv,
                                     float3 oinv, float tbest)
{
    const float x0 = fmaf(nx, inv.x, -oinv.x), x1 = fmaf(fx, inv.x, -oinv.x);
    const float y0 = fmaf(ny, inv.y, -oinv.y), y1 = fmaf(fy, inv.y, -oinv.y);
    const float z0 = fmaf(nz, inv.z, -oinv.z), z1 = fmaf(fz, inv.z, -oinv.z);
    const float tmin = fmaxf(fmaxf(x0, y0), fmaxf(z0, 0.0f));
    const float tmax = fminf(fminf(x1, y1), fminf(z1, tbest));
    return tmin <= tmax ? tmin : __int_as_float(0x7f800000);
}

// sort key of child `slot`: entry distance (>= 0, so its bits are ordered) rounded down to a
// multiple of 4 ulp, slot in the low two bits; kMiss if the box is missed or the slot empty
__device__ inline uint32_t child_key(float t, int32_t code, uint32_t slot)
{
    return (t == __int_as_float(0x7f800000) || code == kBvhEmptySlot) ? kMiss
                                                                      : ((__float_as_uint(t) & ~3u) | slot);
}

// child code named by a sort key's slot (its two low bits), by selects rather than branches
__device__ inline int32_t child_of(const int4& ch, uint32_t key)
{
    const bool odd = (key & 1u) != 0u;
    const int32_t lo = odd ? ch.y : ch.x;
    const int32_t hi = odd ? ch.w : ch.z;
    return (key & 2u) != 0u ? hi : lo;
}

// reciprocal for slab tests only (rounding there is harmless; see the file comment)
__device__ inline float slab_rcp(float a)
{
    return __builtin_amdgcn_rcpf(fabsf(a) < 1e-20f ? copysignf(1e-20f, a) : a);
}

// sorting network: afterwards s0 <= s1 <= s2 <= s3
__device__ inline void sort4(uint32_t& s0, uint32_t& s1, uint32_t& s2, uint32_t& s3)
{
    uint32_t u;
    u = min(s0, s1); s1 = max(s0, s1); s0 = u;
    u = min(s2, s3); s3 = max(s2, s3); s2 = u;
    u = min(s0, s2); s2 = max(s0, s2); s0 = u;
    u = min(s1, s3); s3 = max(s1, s3); s1 = u;
    u = min(s1, s2); s2 = max(s1, s2); s1 = u;
}

}  // namespace rtsdf
