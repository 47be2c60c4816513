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

// Entry parameter of a child box, or +inf if the ray misses it or enters it beyond tbest:
// the slab test with each axis's near and far planes (near = lo where the reciprocal is
// positive, else hi -- the ray's direction signs fix which plane is nearer, so the two
// planes of an axis need no ordering), the interval clipped to [0, tbest].
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

// byte offsets of a node's plane arrays, and of each axis's near planes for a ray whose
// slab reciprocals are `inv` (far = near ^ (lo ^ hi))
constexpr int32_t kLoX = (int32_t)offsetof(Bvh4Node, lox), kLoY = (int32_t)offsetof(Bvh4Node, loy);
constexpr int32_t kLoZ = (int32_t)offsetof(Bvh4Node, loz), kHiX = (int32_t)offsetof(Bvh4Node, hix);
constexpr int32_t kHiY = (int32_t)offsetof(Bvh4Node, hiy), kHiZ = (int32_t)offsetof(Bvh4Node, hiz);

struct NearPlanes {
    int32_t x, y, z;
};

__device__ inline NearPlanes near_planes(float3 inv)
{
    return NearPlanes{inv.x > 0.0f ? kLoX : kHiX, inv.y > 0.0f ? kLoY : kHiY, inv.z > 0.0f ? kLoZ : kHiZ};
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

// the four children's sort keys of `node` (slab test with the ray's near / far planes)
__device__ inline void node_keys(const Bvh4Node* node, NearPlanes np, float3 inv, float3 oinv, float tb,
                                 uint32_t& s0, uint32_t& s1, uint32_t& s2, uint32_t& s3, int4& ch)
{
    const char* N = (const char*)node;
    auto planes = [&](int32_t off) { return *(const float4*)(N + off); };
    const float4 nx = planes(np.x), ny = planes(np.y), nz = planes(np.z);
    const float4 fx = planes(np.x ^ (kLoX ^ kHiX)), fy = planes(np.y ^ (kLoY ^ kHiY)), fz = planes(np.z ^ (kLoZ ^ kHiZ));
    ch = node->child;
    s0 = child_key(box_entry_nf(nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, inv, oinv, tb), ch.x, 0u);
    s1 = child_key(box_entry_nf(nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, inv, oinv, tb), ch.y, 1u);
    s2 = child_key(box_entry_nf(nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, inv, oinv, tb), ch.z, 2u);
    s3 = child_key(box_entry_nf(nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, inv, oinv, tb), ch.w, 3u);
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
