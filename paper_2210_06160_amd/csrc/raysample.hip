// Ray sampling of the masked grid points (section 2.1) against the software LBVH.
//
// One lane per (masked voxel, ray).  Traversal keeps a per-lane stack of (node, entry t)
// and culls a box only when its entry parameter exceeds the best hit so far (ties are
// still visited, because the tie-break is the triangle index).  Box tests may round
// freely: every triangle box is widened by 2*pad while a hit's computed point must lie
// within pad of its triangle's box, so a box holding a hit is never culled and the result
// equals the brute-force least (t, triangle index).
#include "sampling.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 256;
constexpr int kStack = 64;  // radix-tree depth <= 30 code bits + 26 index bits

__device__ inline float box_entry(float4 lo, float4 hi, float3 inv, float3 oinv, float tbest)
{
    const float x0 = fmaf(lo.x, inv.x, -oinv.x), x1 = fmaf(hi.x, inv.x, -oinv.x);
    const float y0 = fmaf(lo.y, inv.y, -oinv.y), y1 = fmaf(hi.y, inv.y, -oinv.y);
    const float z0 = fmaf(lo.z, inv.z, -oinv.z), z1 = fmaf(hi.z, inv.z, -oinv.z);
    const float tmin = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tbest));
    return tmin <= tmax ? tmin : __int_as_float(0x7f800000);
}

__device__ inline float nonzero(float a) { return fabsf(a) < 1e-20f ? copysignf(1e-20f, a) : a; }

struct Closest {
    float t;
    int32_t id;
    bool front;
};

__device__ inline void test_leaf(const BvhTri* __restrict__ tris, int32_t pos, float3 o, float3 w,
                                 Closest& c)
{
    const BvhTri T = tris[pos];
    bool fr = false;
    const float t = hit_triangle(o, w, make_float3(T.v0.x, T.v0.y, T.v0.z),
                                 make_float3(T.e1.x, T.e1.y, T.e1.z), make_float3(T.e2.x, T.e2.y, T.e2.z),
                                 make_float3(T.lo.x, T.lo.y, T.lo.z), make_float3(T.hi.x, T.hi.y, T.hi.z),
                                 fr);
    if (t > 0.0f) {
        const int32_t id = __float_as_int(T.v0.w);
        if (t < c.t || (t == c.t && id < c.id)) {
            c.t = t;
            c.id = id;
            c.front = fr;
        }
    }
}

__device__ Closest closest_hit(const BvhNode* __restrict__ nodes, const BvhTri* __restrict__ tris,
                               int32_t nt, int32_t root, float3 o, float3 w)
{
    const float inf = __int_as_float(0x7f800000);
    Closest c{inf, 0x7FFFFFFF, false};
    if (nt == 0) return c;
    if (root < 0) {
        test_leaf(tris, ~root, o, w, c);
        return c;
    }
    const float3 inv = make_float3(1.0f / nonzero(w.x), 1.0f / nonzero(w.y), 1.0f / nonzero(w.z));
    const float3 oinv = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
    int32_t stk_n[kStack];
    float stk_t[kStack];
    int sp = 0;
    int32_t node = root;
    while (true) {
        const BvhNode n = nodes[node];
        float ta = box_entry(n.a_lo, n.a_hi, inv, oinv, c.t);
        float tb = box_entry(n.b_lo, n.b_hi, inv, oinv, c.t);
        const int32_t ca = __float_as_int(n.a_lo.w), cb = __float_as_int(n.b_lo.w);
        if (ca < 0 && ta != inf) {
            test_leaf(tris, ~ca, o, w, c);
            ta = inf;
        }
        if (cb < 0 && tb != inf) {
            test_leaf(tris, ~cb, o, w, c);
            tb = inf;
        }
        if (ta > c.t) ta = inf;
        if (tb > c.t) tb = inf;
        if (ta != inf && tb != inf) {
            const bool a_first = ta <= tb;
            stk_n[sp] = a_first ? cb : ca;
            stk_t[sp] = a_first ? tb : ta;
            ++sp;
            node = a_first ? ca : cb;
        } else if (ta != inf) {
            node = ca;
        } else if (tb != inf) {
            node = cb;
        } else {
            bool more = false;
            while (sp > 0) {
                --sp;
                if (stk_t[sp] <= c.t) {
                    node = stk_n[sp];
                    more = true;
                    break;
                }
            }
            if (!more) break;
        }
    }
    return c;
}

__global__ __launch_bounds__(kThreads) void k_raysample(const char* __restrict__ bvh, const rtsdf_grid g,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ count_p, int32_t x,
                                                        uint32_t k0, uint32_t k1, uint32_t frame,
                                                        uint32_t obj, float* __restrict__ dmin,
                                                        uint32_t* __restrict__ hits,
                                                        uint64_t* __restrict__ argmin)
{
    const BvhHeader* H = (const BvhHeader*)bvh;
    const int32_t nt = H->nt, root = H->root;
    const BvhNode* nodes = (const BvhNode*)(bvh + 256);
    const BvhTri* tris = (const BvhTri*)(bvh + 256 + sizeof(BvhNode) * (size_t)(nt > 1 ? nt - 1 : 0));
    const int64_t total = (int64_t)(*count_p) * x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total; r += stride) {
        const int64_t b = r / x;
        const uint32_t j = (uint32_t)(r - b * x);
        const int32_t vid = list[b];
        uint32_t i0, i1, i2;
        const float3 o = voxel_centre(g, vid, i0, i1, i2);
        const float3 w = sphere_direction(k0, k1, (uint32_t)vid, frame, j, obj);
        const Closest c = closest_hit(nodes, tris, nt, root, o, w);
        if (c.id != 0x7FFFFFFF) {
            atomicMin((uint32_t*)&dmin[vid], __float_as_uint(c.t));
            atomicAdd(&hits[vid], c.front ? 1u : 65536u);
            if (argmin) {
                const uint64_t rec = ((uint64_t)__float_as_uint(c.t) << 32) | (uint64_t)(frame * (uint32_t)x + j);
                atomicMin((unsigned long long*)&argmin[vid], (unsigned long long)rec);
            }
        }
    }
}

}  // namespace

hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list, const int32_t* count,
                     int64_t capacity, int32_t x, uint64_t key, uint32_t frame, uint32_t obj,
                     float* dmin, uint32_t* hits, uint64_t* argmin, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    const int64_t want = ceil_div(capacity * x, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, persistent_groups(kThreads)));
    hipLaunchKernelGGL(k_raysample, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g, list, count, x,
                       (uint32_t)key, (uint32_t)(key >> 32), frame, obj, dmin, hits, argmin);
    return hipGetLastError();
}

}  // namespace rtsdf
