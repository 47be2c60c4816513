// Ray sampling of the masked grid points (section 2.1) against the software LBVH.
//
// A persistent grid; each lane owns one masked voxel at a time and traces its rays
// j = 0..x-1 one after the other, keeping the minimum distance, hit counts and argmin
// record in registers, and folds them into the voxel's accumulators once at the end
// (min / add are order-free, so the result does not depend on scheduling).  A lane whose
// ray ends starts its next ray at once, and a lane whose voxel is done takes the next
// voxel from a cursor (one atomic per wave per refill), so divergent ray lengths neither
// idle lanes nor leave a tail of busy waves.  The mask list is split into one contiguous
// range per XCD (work-groups are dealt to the 8 XCDs round-robin); a wave takes voxels
// from its own XCD's range first, so list reads and the hierarchy working set stay in
// that XCD's L2, and steals from the other ranges when its own is exhausted.
// The loop touches no cold memory: directions are drawn in registers and accumulators are
// updated with fire-and-forget atomics, because on CDNA loads retire in order and one
// HBM-latency load would stall every later node fetch of the wave.
// Each loop iteration does at most one node visit and one triangle test per lane.
//
// Traversal keeps a per-lane stack of (entry, box entry t) in LDS, spilling to private
// memory past kLdsDepth; entries are internal nodes (>= 0) or leaves (~position).  A box
// is culled only when its entry parameter exceeds the best hit so far (ties are still
// visited, because the tie-break is the triangle index).  Box tests may round freely:
// every triangle box is widened by 2*pad while a hit's computed point must lie within pad
// of its triangle's box, so a box holding a hit is never culled and the result equals the
// brute-force least (t, triangle index).
#include "sampling.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 256;
constexpr int kLdsDepth = 8;
constexpr int kMaxDepth = 64;  // one push per level; radix-tree depth <= 30 code bits + 26 index bits
constexpr int kXcds = 8;
constexpr int32_t kNone = 0x7FFFFFFF;
constexpr int32_t kNoLeaf = 0x7FFFFFFF;

__device__ inline float box_entry(float4 lo, float4 hi, float3 inv, float3 oinv, float tbest)
{
    const float x0 = fmaf(lo.x, inv.x, -oinv.x), x1 = fmaf(hi.x, inv.x, -oinv.x);
    const float y0 = fmaf(lo.y, inv.y, -oinv.y), y1 = fmaf(hi.y, inv.y, -oinv.y);
    const float z0 = fmaf(lo.z, inv.z, -oinv.z), z1 = fmaf(hi.z, inv.z, -oinv.z);
    const float tmin = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tbest));
    return tmin <= tmax ? tmin : __int_as_float(0x7f800000);
}

// reciprocal for slab tests only (rounding there is harmless; see the file comment)
__device__ inline float slab_rcp(float a)
{
    return __builtin_amdgcn_rcpf(fabsf(a) < 1e-20f ? copysignf(1e-20f, a) : a);
}

__device__ inline void test_leaf(const BvhTri* __restrict__ tris, int32_t pos, float3 o, float3 w,
                                 float pad, float& tb, int32_t& bid, bool& bfr)
{
    const float4 a = tris[pos].v0, b = tris[pos].v1, c = tris[pos].v2;
    bool fr = false;
    const float t = hit_triangle(o, w, make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z),
                                 make_float3(c.x, c.y, c.z), pad, fr);
    if (t > 0.0f) {
        const int32_t id = __float_as_int(a.w);
        if (t < tb || (t == tb && id < bid)) {
            tb = t;
            bid = id;
            bfr = fr;
        }
    }
}

// cursors[x] walks XCD x's range [x*count/8, (x+1)*count/8) of the mask list
__global__ void k_cursor_reset(int32_t* cursors)
{
    if (threadIdx.x < kXcds) cursors[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads) void k_raysample(const char* __restrict__ bvh, const rtsdf_grid g,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ count_p, int32_t x,
                                                        uint32_t k0, uint32_t k1, uint32_t frame,
                                                        uint32_t obj, float* __restrict__ dmin,
                                                        uint32_t* __restrict__ hits,
                                                        uint64_t* __restrict__ argmin,
                                                        int32_t* __restrict__ cursors)
{
    __shared__ int32_t s_node[kLdsDepth][kThreads];
    __shared__ float s_t[kLdsDepth][kThreads];
    int32_t p_node[kMaxDepth - kLdsDepth];
    float p_t[kMaxDepth - kLdsDepth];

    const BvhHeader* H = (const BvhHeader*)bvh;
    const int32_t nt = H->nt, root = H->root;
    const float pad = H->pad;
    const BvhNode* __restrict__ nodes = (const BvhNode*)(bvh + 256);
    const BvhTri* __restrict__ tris =
        (const BvhTri*)(bvh + 256 + sizeof(BvhNode) * (size_t)(nt > 1 ? nt - 1 : 0));
    const int32_t count = *count_p;
    const float inf = __int_as_float(0x7f800000);
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const uint32_t code0 = frame * (uint32_t)x;
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    int xcd = (int)(blockIdx.x % kXcds);  // the range this wave takes voxels from
    int tried = 0;                        // ranges found exhausted

    int32_t vid = -1;
    uint32_t j = 0;
    float acc_d = inf;
    uint32_t acc_h = 0;
    uint64_t acc_a = ~0ull;
    float3 o = make_float3(0.f, 0.f, 0.f);
    bool alive = true, active = false;
    float3 w = o, inv = o, oinv = o;
    float tb = inf;
    int32_t bid = kNone;
    bool bfr = false;
    int32_t node = -1, pend = kNoLeaf;
    int sp = 0;

    while (true) {
        // retire a finished ray; fold a finished voxel into its accumulators
        bool need = false;
        if (alive && !active) {
            if (vid >= 0) {
                if (bid != kNone) {
                    acc_d = fminf(acc_d, tb);
                    acc_h += bfr ? 1u : 65536u;
                    const uint64_t rec = ((uint64_t)__float_as_uint(tb) << 32) | (uint64_t)(code0 + j);
                    acc_a = rec < acc_a ? rec : acc_a;
                }
                if (++j == (uint32_t)x) {
                    if (acc_h != 0u) {
                        atomicMin((uint32_t*)&dmin[vid], __float_as_uint(acc_d));
                        atomicAdd(&hits[vid], acc_h);
                        if (argmin) atomicMin((unsigned long long*)&argmin[vid], (unsigned long long)acc_a);
                    }
                    vid = -1;
                }
            }
            need = vid < 0;
        }
        // wave-cooperative refill of voxels from this XCD's range, then the others'
        uint64_t needers = __ballot(need);
        while (needers && tried < kXcds) {
            const int leader = __ffsll((unsigned long long)needers) - 1;
            const int32_t lo = (int32_t)(((int64_t)count * xcd) / kXcds);
            const int32_t hi = (int32_t)(((int64_t)count * (xcd + 1)) / kXcds);
            int32_t base = 0;
            if (lane == leader) base = atomicAdd(&cursors[xcd], (int32_t)__popcll(needers));
            base = __shfl(base, leader) + lo;
            if (need) {
                const int32_t idx = base + (int32_t)__popcll(needers & lt_mask);
                if (idx < hi) {
                    vid = list[idx];
                    need = false;
                    j = 0;
                    acc_d = inf;
                    acc_h = 0u;
                    acc_a = ~0ull;
                    const uint32_t uv = (uint32_t)vid;
                    const uint32_t row = uv / nx;
                    const uint32_t i0 = uv - row * nx, i1 = row % ny, i2 = row / ny;
                    o = make_float3(g.org[0] + g.h * ((float)i0 + 0.5f), g.org[1] + g.h * ((float)i1 + 0.5f),
                                    g.org[2] + g.h * ((float)i2 + 0.5f));
                }
            }
            needers = __ballot(need);
            if (needers) {  // this range is exhausted: move on to the next one
                xcd = (xcd + 1) % kXcds;
                ++tried;
            }
        }
        if (need) alive = false;
        // start the next ray
        if (alive && !active) {
            w = sphere_direction(k0, k1, (uint32_t)vid, frame, j, obj);
            inv = make_float3(slab_rcp(w.x), slab_rcp(w.y), slab_rcp(w.z));
            oinv = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
            tb = inf;
            bid = kNone;
            sp = 0;
            node = -1;
            pend = kNoLeaf;
            if (nt == 1) {
                pend = ~root;
                active = true;
            } else if (nt > 1) {
                node = root;
                active = true;
            }
        }
        if (__ballot(alive) == 0ull) break;
        if (!active) continue;
        // at most one triangle test ...
        if (pend != kNoLeaf) {
            test_leaf(tris, pend, o, w, pad, tb, bid, bfr);
            pend = kNoLeaf;
        }
        // ... and one node visit per iteration
        if (node >= 0) {
            const BvhNode n = nodes[node];
            const float ta = box_entry(n.a_lo, n.a_hi, inv, oinv, tb);
            const float tc = box_entry(n.b_lo, n.b_hi, inv, oinv, tb);
            const int32_t ca = __float_as_int(n.a_lo.w), cc = __float_as_int(n.b_lo.w);
            const bool a_first = ta <= tc;
            const int32_t c1 = a_first ? ca : cc, c2 = a_first ? cc : ca;  // near, far
            const float t1 = a_first ? ta : tc, t2 = a_first ? tc : ta;
            node = -1;
            // the near child goes to `node` (internal) or `pend` (leaf); the far one is pushed.
            // A child that misses has t = inf, so a single hit is always the near one.
            if (t1 != inf) {
                if (c1 >= 0) node = c1;
                else pend = ~c1;
            }
            if (t2 != inf) {
                if (sp < kLdsDepth) {
                    s_node[sp][tid] = c2;
                    s_t[sp][tid] = t2;
                } else {
                    p_node[sp - kLdsDepth] = c2;
                    p_t[sp - kLdsDepth] = t2;
                }
                ++sp;
            }
        }
        // refill node / pending leaf from the stack
        while (node < 0 && sp > 0) {
            const int top = sp - 1;
            int32_t e;
            float t;
            if (top < kLdsDepth) {
                e = s_node[top][tid];
                t = s_t[top][tid];
            } else {
                e = p_node[top - kLdsDepth];
                t = p_t[top - kLdsDepth];
            }
            if (t > tb) {
                sp = top;
                continue;
            }
            if (e >= 0) {
                node = e;
                sp = top;
            } else if (pend == kNoLeaf) {
                pend = ~e;
                sp = top;
            } else {
                break;
            }
        }
        if (node < 0 && pend == kNoLeaf && sp == 0) active = false;
    }
}

}  // namespace

size_t raysample_work_bytes(int64_t, int32_t) { return 256; }

hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list, const int32_t* count,
                     int64_t capacity, int32_t x, uint64_t key, uint32_t frame, uint32_t obj,
                     float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    int32_t* cursors = (int32_t*)work;
    hipLaunchKernelGGL(k_cursor_reset, dim3(1), dim3(64), 0, s, cursors);
    // exactly the resident grid: more groups would only start after others finish
    static int resident = 0;
    if (resident == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raysample, kThreads, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        resident = per_cu * cus;
    }
    const int64_t want = ceil_div(capacity, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(kXcds, std::min<int64_t>(want, resident));
    hipLaunchKernelGGL(k_raysample, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g, list, count, x,
                       (uint32_t)key, (uint32_t)(key >> 32), frame, obj, dmin, hits, argmin, cursors);
    return hipGetLastError();
}

}  // namespace rtsdf
