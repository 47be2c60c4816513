// Derivative of the running-minimum fine field with respect to vertex positions (section
// 2.1 ray sampling, differentiated with the discrete state held fixed).
//
// A masked grid point with hits holds fine = sign * t - bias, where t is the distance along
// the ray its argmin record names (frame * x + j, with t's bits above).  The ray is rebuilt
// from that record (same counter-based direction as the forward) and traced again to its
// closest hit, the least (t, triangle index), which by the exact-culling argument of the
// traversal helpers is the triangle the forward found.  Moving vertex k of that triangle by
// d moves the plane at the hit point by b_k d, so dt/dv_k = b_k n / (n . w).
//
// One lane per listed grid point (grid-stride); a closest-hit traversal of the 4-wide
// hierarchy with a per-lane stack in LDS that spills to private memory, in the iteration
// structure of ray sampling; the gradient is scattered to the three vertices with binary32
// atomic adds.  Device-scope atomics are the slow part (they serialise at the memory side),
// and neighbouring list entries mostly hit the same triangles (their closest rays run to the
// nearest surface), so the lanes of a wave that hit one triangle first sum their nine values
// in LDS and one of them issues the triangle's nine atomics.
#include "traverse.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 128;
constexpr int kLdsDepth = 8;

// kBatch: list entries index concatenated grids; each voxel's object supplies its grid, its
// hierarchy, the counter's object word and the base of its vertices and triangles.
template <bool kBatch>
__global__ __launch_bounds__(kThreads) void k_sdf_backward(
    const char* __restrict__ bvh, const rtsdf_grid g, const int32_t* __restrict__ list,
    const int32_t* __restrict__ count_p, const float* __restrict__ grad_fine,
    const uint32_t* __restrict__ hits, const uint64_t* __restrict__ argmin,
    const int32_t* __restrict__ tri_index, int32_t x, uint32_t k0, uint32_t k1, uint32_t obj,
    float* __restrict__ grad_verts, const char* plan, int32_t nobj)
{
    __shared__ uint64_t s_stk[kLdsDepth][kThreads];  // child keys: (entry t bits << 32) | code
    __shared__ float s_acc[9][kThreads];             // a group leader's sums (3 vertices x 3)
    // spilled entries as two 32-bit arrays: a 64-bit array would let the compiler merge its
    // reads with the LDS reads into one flat load, which occupies the vector-memory path
    // even for LDS addresses
    uint32_t p_t[kMaxStack - kLdsDepth];
    uint32_t p_code[kMaxStack - kLdsDepth];

    int32_t nt = 0, root = 0;
    bool deep = false;  // the hierarchy is too deep for the stack: test every triangle
    float pad = 0.0f;
    const char* __restrict__ nodes = nullptr;
    const BvhTri* __restrict__ tris = nullptr;
    auto use_bvh = [&](const char* b) {
        const BvhHeader* H = (const BvhHeader*)b;
        nt = H->nt;
        root = H->root;
        deep = bvh_too_deep(H->depth);
        pad = H->pad;
        nodes = b + 256;
        tris = (const BvhTri*)(b + 256 + sizeof(Bvh4Node) * (size_t)(nt > 1 ? nt - 1 : 1));
    };
    if (!kBatch) {
        use_bvh(bvh);
        if (nt == 0) return;
    }
    const int32_t count = *count_p;
    const float inf = __int_as_float(0x7f800000);
    const int tid = threadIdx.x;

    for (int64_t q = (int64_t)blockIdx.x * kThreads + tid; q < count; q += (int64_t)gridDim.x * kThreads) {
        const int32_t vid = list[q];
        const uint32_t hc = hits[vid];
        const float gf = grad_fine[vid];
        if (hc == 0u || gf == 0.0f) continue;
        rtsdf_grid lg = g;
        uint32_t lvid = (uint32_t)vid, lobj = obj;
        const int32_t* ltri = tri_index;
        float* lgv = grad_verts;
        if (kBatch) {
            const BatchView bv = batch_view(plan, nobj);
            const int32_t oi = find_object(bv.vox_prefix, nobj, (int64_t)vid);
            const BatchObject& ob = bv.obj[oi];
            lvid = (uint32_t)(vid - ob.vox_off);
            lg = ob.g;
            lobj = (uint32_t)oi;
            ltri = tri_index + 3 * (int64_t)ob.tri_off;
            lgv = grad_verts + 3 * (int64_t)ob.vert_off;
            use_bvh(bvh + ob.bvh_off);
            if (nt == 0) continue;
        }
        const uint32_t code = (uint32_t)argmin[vid];
        const uint32_t frame = code / (uint32_t)x, j = code - frame * (uint32_t)x;
        uint32_t ci, cj, ck;
        const float3 o = voxel_centre(lg, lvid, ci, cj, ck);
        const float3 w = sphere_direction(k0, k1, lvid, frame, j, lobj);
        const float3 inv = make_float3(slab_rcp(w.x), slab_rcp(w.y), slab_rcp(w.z));
        const float3 oinv = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
        const NearPlanes np = near_planes(inv);

        float tb = inf;
        int32_t bid = kNone, bpos = -1;
        int sp = 0;
        // (sp < kMaxStack always holds: deeper hierarchies are not traversed; the test keeps
        // the private arrays in bounds regardless)
        auto push = [&](uint64_t word) {
            if (sp < kLdsDepth) {
                s_stk[sp][tid] = word;
            } else if (sp < kMaxStack) {
                p_t[sp - kLdsDepth] = (uint32_t)(word >> 32);
                p_code[sp - kLdsDepth] = (uint32_t)word;
            }
            sp = min(sp + 1, kMaxStack);
        };
        // The traversal loop of ray sampling: per iteration at most one triangle test and one
        // node visit, at most two stack pops, and up to two pending leaf ranges (so that the
        // lanes of a wave do similar work in every iteration).
        int32_t node = -1, pfirst = 0, pcount = 0, pfirst2 = 0, pcount2 = 0;
        if (root >= 0 && !deep) {
            node = root;
        } else if (root >= 0) {
            pcount = nt;  // every triangle, in sorted order: the same closest hit
        } else {
            pfirst = leaf_first(root);
            pcount = leaf_count(root);
        }
        auto take_leaf = [&](int32_t code) {  // false: both pending ranges are in use
            if (pcount == 0) {
                pfirst = leaf_first(code);
                pcount = leaf_count(code);
            } else if (pcount2 == 0) {
                pfirst2 = leaf_first(code);
                pcount2 = leaf_count(code);
            } else {
                return false;
            }
            return true;
        };
        while (node >= 0 || pcount > 0 || sp > 0) {
            if (pcount > 0) {
                const float4 a = tris[pfirst].v0, b = tris[pfirst].v1, c = tris[pfirst].v2;
                bool fr = false;
                const float t = hit_triangle(o, w, make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z),
                                             make_float3(c.x, c.y, c.z), pad, fr);
                const int32_t id = __float_as_int(a.w);
                if (t > 0.0f && (t < tb || (t == tb && id < bid))) {
                    tb = t;
                    bid = id;
                    bpos = pfirst;
                }
                ++pfirst;
                if (--pcount == 0) {
                    pfirst = pfirst2;
                    pcount = pcount2;
                    pcount2 = 0;
                }
            }
            if (node >= 0) {
                ChildKey s0, s1, s2, s3;
                node_keys(fetch_node(nodes, (uint32_t)node), np, inv, oinv, tb, s0, s1, s2, s3);
                sort4(s0, s1, s2, s3);
                if (entered(s3)) push(stack_word(s3));
                if (entered(s2)) push(stack_word(s2));
                if (entered(s1)) push(stack_word(s1));
                node = -1;
                if (entered(s0)) {
                    if (s0.code >= 0) {
                        node = s0.code;
                    } else if (!take_leaf(s0.code)) {
                        push(stack_word(s0));
                    }
                }
            }
            // next entries whose boxes may still hold a hit no farther than the best so far
            for (int trips = 0; node < 0 && sp > 0 && trips < 2; ++trips) {
                const int top = sp - 1;
                uint64_t word;
                if (top < kLdsDepth) {
                    word = s_stk[top][tid];
                } else {
                    word = ((uint64_t)p_t[top - kLdsDepth] << 32) | p_code[top - kLdsDepth];
                }
                if (word_t(word) > tb) {
                    sp = top;
                    continue;
                }
                const int32_t e = word_code(word);
                if (e >= 0) {
                    node = e;
                } else if (!take_leaf(e)) {
                    break;
                }
                sp = top;
            }
        }
        // lanes whose ray hit nothing (bpos < 0) stay for the wave's aggregation below
        const bool valid = bpos >= 0;
        float val[9];
        int32_t gtri = -1;                 // the hit triangle across the batch
        const int32_t* tv = nullptr;
        if (valid) {
            const float4 a = tris[bpos].v0, b = tris[bpos].v1, c = tris[bpos].v2;
            const float3 v0 = make_float3(a.x, a.y, a.z);
            const float3 e1 = make_float3(b.x - a.x, b.y - a.y, b.z - a.z);
            const float3 e2 = make_float3(c.x - a.x, c.y - a.y, c.z - a.z);
            const float3 n = cross3(e1, e2);
            const float nw = dot3(n, w);
            // barycentrics of the hit (Moller-Trumbore u, v)
            const float3 P = cross3(w, e2);
            const float inv_det = 1.0f / dot3(e1, P);
            const float3 T = make_float3(o.x - v0.x, o.y - v0.y, o.z - v0.z);
            const float u = dot3(T, P) * inv_det;
            const float v = dot3(w, cross3(T, e1)) * inv_det;
            const float bary[3] = {(1.0f - u) - v, u, v};
            const float sign = (hc >> 16) > (hc & 0xFFFFu) ? -1.0f : 1.0f;
            const float scale = gf * sign / nw;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float sk = scale * bary[k];
                val[3 * k + 0] = sk * n.x;
                val[3 * k + 1] = sk * n.y;
                val[3 * k + 2] = sk * n.z;
            }
            gtri = (int32_t)((ltri - tri_index) / 3) + bid;
            tv = ltri + 3 * (int64_t)bid;
        }
        // group the wave's lanes by hit triangle: each lane learns its group's first lane
        const int lane = tid & (kWave - 1), wbase = tid - lane;
        int leader = lane;
        uint64_t pending = __ballot(valid);
        while (pending != 0ull) {
            const int l = __ffsll((long long)pending) - 1;
            const int32_t kl = __shfl(gtri, l);
            const bool mine = valid && gtri == kl;
            if (mine) leader = l;
            pending &= ~__ballot(mine);
        }
        // leaders clear their slots, every member adds into its leader's (LDS atomics; LDS
        // operations of one wave complete in order), leaders scatter the sums
        if (valid && leader == lane)
            for (int i = 0; i < 9; ++i) s_acc[i][tid] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        if (valid)
            for (int i = 0; i < 9; ++i) atomicAdd(&s_acc[i][wbase + leader], val[i]);
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __builtin_amdgcn_wave_barrier();
        if (valid && leader == lane) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float* gv = lgv + 3 * (int64_t)tv[k];
                unsafeAtomicAdd(gv + 0, s_acc[3 * k + 0][tid]);
                unsafeAtomicAdd(gv + 1, s_acc[3 * k + 1][tid]);
                unsafeAtomicAdd(gv + 2, s_acc[3 * k + 2][tid]);
            }
        }
    }
}

}  // namespace

hipError_t sdf_backward(const float* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                        const int32_t* list, const int32_t* count, int64_t capacity, const void* bvh,
                        const int32_t* tris, const rtsdf_grid& g, int32_t x, uint64_t key, uint32_t obj,
                        float* grad_verts, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    const int64_t want = ceil_div(capacity, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, persistent_groups(kThreads)));
    hipLaunchKernelGGL(k_sdf_backward<false>, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g, list, count,
                       grad_fine, hits, argmin, tris, x, (uint32_t)key, (uint32_t)(key >> 32), obj, grad_verts,
                       nullptr, 0);
    return hipGetLastError();
}

hipError_t sdf_backward_batched(const BatchView& hv, const void* dplan, const float* grad_fine,
                                const uint32_t* hits, const uint64_t* argmin, const int32_t* list,
                                const int32_t* count, int64_t capacity, const void* bvh, const int32_t* tris,
                                int32_t x, uint64_t key, float* grad_verts, hipStream_t s)
{
    if (capacity <= 0 || hv.h->total_tris == 0) return hipSuccess;
    const int64_t want = ceil_div(capacity, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, persistent_groups(kThreads)));
    const rtsdf_grid g0 = hv.obj[0].g;  // unused in batch mode
    hipLaunchKernelGGL(k_sdf_backward<true>, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g0, list, count,
                       grad_fine, hits, argmin, tris, x, (uint32_t)key, (uint32_t)(key >> 32), 0u, grad_verts,
                       (const char*)dplan, hv.h->nobj);
    return hipGetLastError();
}

}  // namespace rtsdf
