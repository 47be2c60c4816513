// Helpers shared by the kernels that trace rays through the 4-wide hierarchy written by
// lbvh.hip: the slab test of a quantised child box and the sort key of a child (the stack
// bound and the depth rule are in layout.h).  Box tests may round freely: every triangle box is widened
// by 2*pad, the quantised boxes contain those, and a hit's computed point must lie within
// pad of its triangle's box, so a box holding a hit is never culled and traversal returns
// the brute-force least (t, index).
#pragma once

#include "sampling.h"

namespace rtsdf {

constexpr int32_t kNone = 0x7FFFFFFF;

// Per-ray choice of each axis's near planes: the low planes where the slab reciprocal is
// positive, else the high ones (the direction's signs fix which plane is nearer, so the two
// planes of an axis need no ordering).
struct NearPlanes {
    bool x, y, z;
};

__device__ inline NearPlanes near_planes(float3 inv)
{
    return NearPlanes{inv.x > 0.0f, inv.y > 0.0f, inv.z > 0.0f};
}

// A child's key: its entry parameter's bits (>= 0, so they order as unsigned) and its code;
// on the traversal stack the two form one 64-bit word (t bits high).  A box the ray misses,
// or enters beyond tbest, and an unused slot, get t bits kMissT and sort after every entered
// box.
constexpr uint32_t kMissT = 0xFFFFFFFFu;
struct ChildKey {
    uint32_t t;
    int32_t code;
};
__device__ inline bool entered(const ChildKey& k) { return k.t != kMissT; }
__device__ inline uint64_t stack_word(const ChildKey& k) { return ((uint64_t)k.t << 32) | (uint32_t)k.code; }
__device__ inline float word_t(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32)); }
__device__ inline int32_t word_code(uint64_t w) { return (int32_t)(uint32_t)w; }

// Slab test of one child box given its near and far planes on each axis as parameters
// t = q * a + b of the quantised plane q (see node_keys), the interval clipped to
// [0, tbest]; returns the child's key.
__device__ inline ChildKey box_key(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t fx, uint32_t fy, uint32_t fz,
                                   float3 a, float3 b, float tbest, int32_t code)
{
    const float x0 = fmaf((float)nx, a.x, b.x), x1 = fmaf((float)fx, a.x, b.x);
    const float y0 = fmaf((float)ny, a.y, b.y), y1 = fmaf((float)fy, a.y, b.y);
    const float z0 = fmaf((float)nz, a.z, b.z), z1 = fmaf((float)fz, a.z, b.z);
    const float tmin = fmaxf(fmaxf(x0, y0), fmaxf(z0, 0.0f));
    const float tmax = fminf(fminf(x1, y1), fminf(z1, tbest));
    return ChildKey{(tmin <= tmax && code != kBvhEmptySlot) ? __float_as_uint(tmin) : kMissT, code};
}

// reciprocal for slab tests only (rounding there is harmless; see the file comment)
__device__ inline float slab_rcp(float a)
{
    return __builtin_amdgcn_rcpf(fabsf(a) < 1e-20f ? copysignf(1e-20f, a) : a);
}

// What a ray reads of a node: origin and step exponents, child codes, and the quantised
// planes (lo x, lo y, lo z, hi x | hi y, hi z), in four loads.
struct NodeFetch {
    float4 hdr;
    int4 ch;
    uint4 qa;
    uint2 qb;
};

// Reads node `node` of the node array at `nodes` (byte offsets are 32-bit: a hierarchy
// holds fewer than 2^26 nodes).
__device__ inline NodeFetch fetch_node(const char* __restrict__ nodes, uint32_t node)
{
    const uint32_t b = node << 6;
    NodeFetch f;
    f.hdr = *(const float4*)(nodes + b);
    f.ch = *(const int4*)(nodes + b + offsetof(Bvh4Node, child));
    f.qa = *(const uint4*)(nodes + b + offsetof(Bvh4Node, lo));
    f.qb = *(const uint2*)(nodes + b + offsetof(Bvh4Node, hi[1]));
    return f;
}

// byte q of a quantised plane word
__device__ inline uint32_t plane_byte(uint32_t w, int q) { return (w >> (8 * q)) & 0xFFu; }

// The step 2^(e - 127) of the biased exponent in bits [sh, sh + 8) of e.
__device__ inline float axis_step(uint32_t e, int sh) { return __uint_as_float(((e >> sh) & 0xFFu) << 23); }

// The four children's keys of a fetched node.  On axis a a quantised plane q lies at
// c_a + q s_a (c: the node's low corner), which the ray from p reaches at parameter
// (c_a + q s_a - p_a) inv_a = q (s_a inv_a) + (c_a inv_a - p_a inv_a); oinv holds p inv.
__device__ inline void node_keys(const NodeFetch& f, const NearPlanes& np, float3 inv, float3 oinv, float tb,
                                 ChildKey& s0, ChildKey& s1, ChildKey& s2, ChildKey& s3)
{
    const uint32_t e = __float_as_uint(f.hdr.w);
    const float3 a = make_float3(axis_step(e, 0) * inv.x, axis_step(e, 8) * inv.y, axis_step(e, 16) * inv.z);
    const float3 b = make_float3(fmaf(f.hdr.x, inv.x, -oinv.x), fmaf(f.hdr.y, inv.y, -oinv.y),
                                 fmaf(f.hdr.z, inv.z, -oinv.z));
    const uint32_t lx = f.qa.x, ly = f.qa.y, lz = f.qa.z, hx = f.qa.w, hy = f.qb.x, hz = f.qb.y;
    const uint32_t nx = np.x ? lx : hx, fx = np.x ? hx : lx;
    const uint32_t ny = np.y ? ly : hy, fy = np.y ? hy : ly;
    const uint32_t nz = np.z ? lz : hz, fz = np.z ? hz : lz;
    auto key = [&](int q, int32_t code) {
        return box_key(plane_byte(nx, q), plane_byte(ny, q), plane_byte(nz, q), plane_byte(fx, q), plane_byte(fy, q),
                       plane_byte(fz, q), a, b, tb, code);
    };
    s0 = key(0, f.ch.x);
    s1 = key(1, f.ch.y);
    s2 = key(2, f.ch.z);
    s3 = key(3, f.ch.w);
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
