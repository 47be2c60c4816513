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

// byte offsets of a node's plane arrays (all below 128, the node's size and alignment)
constexpr uint32_t kLoX = (uint32_t)offsetof(Bvh4Node, lox), kLoY = (uint32_t)offsetof(Bvh4Node, loy);
constexpr uint32_t kLoZ = (uint32_t)offsetof(Bvh4Node, loz), kHiX = (uint32_t)offsetof(Bvh4Node, hix);
constexpr uint32_t kHiY = (uint32_t)offsetof(Bvh4Node, hiy), kHiZ = (uint32_t)offsetof(Bvh4Node, hiz);
constexpr uint32_t kChild = (uint32_t)offsetof(Bvh4Node, child);
static_assert(sizeof(Bvh4Node) == 128 && kChild < 128, "node byte offsets are node * 128 | field");

// Per-ray byte offsets of each axis's near planes: lo where the slab reciprocal is
// positive, else hi (the direction's signs fix which plane is nearer, so the two planes of
// an axis need no ordering); an axis's far planes are at near ^ (lo ^ hi).
struct NearPlanes {
    uint32_t x, y, z;
};

__device__ inline NearPlanes near_planes(float3 inv)
{
    return NearPlanes{inv.x > 0.0f ? kLoX : kHiX, inv.y > 0.0f ? kLoY : kHiY, inv.z > 0.0f ? kLoZ : kHiZ};
}

// A child's key: its entry parameter's bits (>= 0, so they order as unsigned) and its code;
// on the traversal stack the two form one 64-bit word (t bits high).  A box the ray misses,
// or enters beyond tbest, gets t bits kMissT and sorts after every entered box.  Unused slots
// hold the empty box lo = +inf, hi = -inf (entry +inf, exit -inf for every direction), so
// the slab test alone rejects them.
constexpr uint32_t kMissT = 0xFFFFFFFFu;
struct ChildKey {
    uint32_t t;
    int32_t code;
};
__device__ inline bool entered(const ChildKey& k) { return k.t != kMissT; }
__device__ inline uint64_t stack_word(const ChildKey& k) { return ((uint64_t)k.t << 32) | (uint32_t)k.code; }
__device__ inline float word_t(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32)); }
__device__ inline int32_t word_code(uint64_t w) { return (int32_t)(uint32_t)w; }

// Slab test of one child box with the ray's near and far planes, the interval clipped to
// [0, tbest]; returns the child's key.
__device__ inline ChildKey box_key(float nx, float ny, float nz, float fx, float fy, float fz, float3 inv,
                                   float3 oinv, float tbest, int32_t code)
{
    const float x0 = fmaf(nx, inv.x, -oinv.x), x1 = fmaf(fx, inv.x, -oinv.x);
    const float y0 = fmaf(ny, inv.y, -oinv.y), y1 = fmaf(fy, inv.y, -oinv.y);
    const float z0 = fmaf(nz, inv.z, -oinv.z), z1 = fmaf(fz, inv.z, -oinv.z);
    const float tmin = fmaxf(fmaxf(x0, y0), fmaxf(z0, 0.0f));
    const float tmax = fminf(fminf(x1, y1), fminf(z1, tbest));
    return ChildKey{tmin <= tmax ? __float_as_uint(tmin) : kMissT, code};
}

// reciprocal for slab tests only (rounding there is harmless; see the file comment)
__device__ inline float slab_rcp(float a)
{
    return __builtin_amdgcn_rcpf(fabsf(a) < 1e-20f ? copysignf(1e-20f, a) : a);
}

// What a ray reads of a node: its near and far planes per axis and the child codes.
struct NodeFetch {
    float4 nx, ny, nz, fx, fy, fz;
    int4 ch;
};

// Reads node `node` of the node array at `nodes` (byte offsets are 32-bit: a hierarchy
// holds fewer than 2^25 nodes).
__device__ inline NodeFetch fetch_node(const char* __restrict__ nodes, uint32_t node, const NearPlanes& np)
{
    const uint32_t b = node << 7;
    const uint32_t ax = b | np.x, ay = b | np.y, az = b | np.z;
    auto planes = [&](uint32_t off) { return *(const float4*)(nodes + off); };
    NodeFetch f;
    f.nx = planes(ax);
    f.ny = planes(ay);
    f.nz = planes(az);
    f.fx = planes(ax ^ (kLoX ^ kHiX));
    f.fy = planes(ay ^ (kLoY ^ kHiY));
    f.fz = planes(az ^ (kLoZ ^ kHiZ));
    f.ch = *(const int4*)(nodes + b + kChild);
    return f;
}

// The four children's keys of a fetched node.
__device__ inline void node_keys(const NodeFetch& f, float3 inv, float3 oinv, float tb, ChildKey& s0, ChildKey& s1,
                                 ChildKey& s2, ChildKey& s3)
{
    s0 = box_key(f.nx.x, f.ny.x, f.nz.x, f.fx.x, f.fy.x, f.fz.x, inv, oinv, tb, f.ch.x);
    s1 = box_key(f.nx.y, f.ny.y, f.nz.y, f.fx.y, f.fy.y, f.fz.y, inv, oinv, tb, f.ch.y);
    s2 = box_key(f.nx.z, f.ny.z, f.nz.z, f.fx.z, f.fy.z, f.fz.z, inv, oinv, tb, f.ch.z);
    s3 = box_key(f.nx.w, f.ny.w, f.nz.w, f.fx.w, f.fy.w, f.fz.w, inv, oinv, tb, f.ch.w);
}

// sorting network on the keys' entry parameters: afterwards s0 .. s3 enter in increasing
// order (entered boxes first); children that enter at the same t keep a fixed order
__device__ inline void sort4(ChildKey& s0, ChildKey& s1, ChildKey& s2, ChildKey& s3)
{
    auto cas = [](ChildKey& a, ChildKey& b) {
        const bool sw = b.t < a.t;
        const ChildKey lo{sw ? b.t : a.t, sw ? b.code : a.code};
        b = ChildKey{sw ? a.t : b.t, sw ? a.code : b.code};
        a = lo;
    };
    cas(s0, s1);
    cas(s2, s3);
    cas(s0, s2);
    cas(s1, s3);
    cas(s1, s2);
}

}  // namespace rtsdf
