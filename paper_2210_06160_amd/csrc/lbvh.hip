// Software BVH for the ray sampling of section 2.1 (the paper relies on the graphics
// driver's hierarchy and RT cores; gfx950 has neither), built for one object or for every
// object of a batch at once.
//
//   centroid bounds per object (atomic min/max on order-preserving float encodings)
//   -> 30-bit Morton code per triangle centroid
//   -> stable LSD radix sort of (code, triangle) in four 8-bit passes, segmented: every
//      sort tile belongs to one object and the digit counts are laid out
//      [object][digit][tile], so one global exclusive scan gives every element a
//      destination inside its own object's range
//   -> a binary tree per object, either
//        LBVH: the binary radix tree over the sorted codes (Karras 2012, "Maximizing
//              parallelism in the construction of BVHs, octrees, and k-d trees"; equal
//              codes are ordered by position) and a bottom-up refit, or
//        PLOC: parallel locally-ordered clustering (Meister & Bittner 2018): the clusters,
//              in Morton order, repeatedly merge with their mutual nearest neighbour by
//              merged-box surface area within +-kPlocRadius positions; kPlocWide
//              iterations run over all objects with one launch per phase, then one
//              work-group per object finishes its remaining clusters.  The binary nodes
//              are numbered from the last merge (the root, 0) backwards, and each leaf
//              walks to the root to find its depth-first position, so that every subtree
//              covers consecutive triangles.
//   -> collapse into the 4-wide hierarchy that traversal reads.
// Boxes are widened so traversal is exact (see traverse.h); the tree only changes speed.
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = kBvhSortTile / kSortThreads;
constexpr int kPlocRadius = RTSDF_PLOC_RADIUS;
constexpr int kPlocThreads = 256;
constexpr int kPlocWide = RTSDF_PLOC_WIDE;
constexpr int kFinishThreads = 1024;

// ---- objects ------------------------------------------------------------------------------
// One object: its triangles [tri_off, tri_off + nt) of the concatenated arrays (positions of
// the sorted arrays, binary nodes and per-triangle state use the same range), its vertex
// base, its first sort tile, its blob and its hit padding.
struct Seg {
    int32_t o, tri_off, nt, vert_off, tile_off;
    int64_t bvh_off;
    float pad;
};

struct Args {       // single object: the fields below; batch: the device plan
    const char* plan;
    int32_t nobj;
    int32_t nt;
    float pad;
};

template <bool kBatch>
__device__ inline Seg seg_of_obj(const Args& a, int32_t o)
{
    if (!kBatch) return Seg{0, 0, a.nt, 0, 0, 0, a.pad};
    const BatchView v = batch_view(a.plan, a.nobj);
    const BatchObject& b = v.obj[o];
    return Seg{o, b.tri_off, b.nt, b.vert_off, b.tile_off, b.bvh_off, b.g.h * (1.0f / 256.0f)};
}

template <bool kBatch>
__device__ inline Seg seg_of_tri(const Args& a, int32_t t)
{
    if (!kBatch) return seg_of_obj<false>(a, 0);
    const BatchView v = batch_view(a.plan, a.nobj);
    return seg_of_obj<true>(a, find_object(v.tri_prefix, a.nobj, t));
}

template <bool kBatch>
__device__ inline Seg seg_of_tile(const Args& a, int32_t tile)
{
    if (!kBatch) return seg_of_obj<false>(a, 0);
    const BatchView v = batch_view(a.plan, a.nobj);
    int32_t lo = 0, hi = a.nobj - 1;  // last object whose first tile is <= tile
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (v.obj[mid].tile_off <= tile) lo = mid;
        else hi = mid - 1;
    }
    return seg_of_obj<true>(a, lo);
}

__device__ inline int32_t tiles_of(int32_t nt) { return (nt + kBvhSortTile - 1) / kBvhSortTile; }

__device__ inline uint32_t f2o(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float o2f(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ inline float3 tri_centroid(const float* __restrict__ v, const int32_t* __restrict__ t, int32_t i)
{
    const int64_t a = t[3 * (int64_t)i], b = t[3 * (int64_t)i + 1], c = t[3 * (int64_t)i + 2];
    const float third = 1.0f / 3.0f;
    return make_float3((v[3 * a] + v[3 * b] + v[3 * c]) * third, (v[3 * a + 1] + v[3 * b + 1] + v[3 * c + 1]) * third,
                       (v[3 * a + 2] + v[3 * b + 2] + v[3 * c + 2]) * third);
}

// triangle box widened by 2 pad (culling stays exact, see traverse.h)
__device__ inline void tri_box(const float* __restrict__ v, const int32_t* __restrict__ t, int32_t i, float pad,
                               float3& lo, float3& hi)
{
    const int64_t ia = t[3 * (int64_t)i], ib = t[3 * (int64_t)i + 1], ic = t[3 * (int64_t)i + 2];
    const float pad2 = 2.0f * pad;
    lo = make_float3(fminf(fminf(v[3 * ia], v[3 * ib]), v[3 * ic]) - pad2,
                     fminf(fminf(v[3 * ia + 1], v[3 * ib + 1]), v[3 * ic + 1]) - pad2,
                     fminf(fminf(v[3 * ia + 2], v[3 * ib + 2]), v[3 * ic + 2]) - pad2);
    hi = make_float3(fmaxf(fmaxf(v[3 * ia], v[3 * ib]), v[3 * ic]) + pad2,
                     fmaxf(fmaxf(v[3 * ia + 1], v[3 * ib + 1]), v[3 * ic + 1]) + pad2,
                     fmaxf(fmaxf(v[3 * ia + 2], v[3 * ib + 2]), v[3 * ic + 2]) + pad2);
}

// ---- per-object set-up, bounds, Morton codes ------------------------------------------------
template <bool kBatch>
__global__ void k_init(Args a, uint32_t* __restrict__ bounds, int32_t* __restrict__ cseg, int32_t* __restrict__ base,
                       int64_t total)
{
    const int32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nobj = kBatch ? a.nobj : 1;
    if (o < nobj) {
        for (int q = 0; q < 3; ++q) {
            bounds[6 * o + q] = 0xFFFFFFFFu;  // running min (encoded)
            bounds[6 * o + 3 + q] = 0u;       // running max (encoded)
        }
        cseg[o] = seg_of_obj<kBatch>(a, o).tri_off;
        base[o] = 0;
    }
    if (o == 0) cseg[nobj] = (int32_t)total;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Per-object centroid bounds.  A work-group reduces kBoundsItems x 256 consecutive
// triangles (lane registers, then the wave, then the group through LDS) and updates an
// object's six bound words once: atomics on one address serialise across the chip, and one
// set per wave cost a few hundred serialised updates per large object.  A thread whose
// triangles cross into another object (rare: objects hold thousands) updates the first
// object's bounds itself; a wave or group spanning objects falls back to one set per lane.
constexpr int kBoundsItems = 16;

template <bool kBatch>
__global__ __launch_bounds__(256) void k_bounds(Args a, const float* __restrict__ v, const int32_t* __restrict__ t,
                                                int32_t total, uint32_t* __restrict__ bounds)
{
    __shared__ uint32_t part[256 / kWave][6];
    __shared__ int32_t part_o[256 / kWave];
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
    int32_t o = -1;  // object of the triangles in mn / mx (-1: none yet)
    auto update = [&](int32_t obj) {
        for (int q = 0; q < 3; ++q) {
            atomicMin(&bounds[6 * obj + q], mn[q]);
            atomicMax(&bounds[6 * obj + 3 + q], mx[q]);
        }
    };
    const int64_t first = (int64_t)blockIdx.x * 256 * kBoundsItems + threadIdx.x;
    for (int j = 0; j < kBoundsItems; ++j) {
        const int64_t i = first + (int64_t)j * 256;
        if (i >= total) break;
        const Seg s = seg_of_tri<kBatch>(a, (int32_t)i);
        if (s.o != o) {
            if (o >= 0) update(o);
            o = s.o;
            for (int q = 0; q < 3; ++q) {
                mn[q] = 0xFFFFFFFFu;
                mx[q] = 0u;
            }
        }
        const float3 c = tri_centroid(v + 3 * (int64_t)s.vert_off, t + 3 * (int64_t)s.tri_off, (int32_t)i - s.tri_off);
        const uint32_t e[3] = {f2o(c.x), f2o(c.y), f2o(c.z)};
        for (int q = 0; q < 3; ++q) {
            mn[q] = min(mn[q], e[q]);
            mx[q] = max(mx[q], e[q]);
        }
    }
    // lanes without triangles (o < 0) hold the neutral values; the wave reduces when every
    // other lane ends in one object
    const uint64_t has = __ballot(o >= 0);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    int32_t wo = -1;
    if (has != 0ull) {
        const int32_t o0 = __shfl(o, __ffsll((long long)has) - 1);
        if (__ballot(o >= 0 && o != o0) == 0ull) {
            for (int d = kWave / 2; d > 0; d >>= 1)
                for (int q = 0; q < 3; ++q) {
                    mn[q] = min(mn[q], (uint32_t)__shfl_xor((int)mn[q], d, kWave));
                    mx[q] = max(mx[q], (uint32_t)__shfl_xor((int)mx[q], d, kWave));
                }
            wo = o0;
        } else if (o >= 0) {
            update(o);  // a wave spanning objects
        }
    }
    if (lane == 0) {
        part_o[wave] = wo;
        for (int q = 0; q < 3; ++q) {
            part[wave][q] = mn[q];
            part[wave][3 + q] = mx[q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t go = -1;
        bool one = true;
        for (int w = 0; w < 256 / kWave; ++w) {
            if (part_o[w] < 0) continue;
            if (go < 0) go = part_o[w];
            else if (part_o[w] != go) one = false;
        }
        if (go >= 0 && one) {
            // only the waves that reduced to one object (part_o >= 0) are merged
            uint32_t gmn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, gmx[3] = {0u, 0u, 0u};
            for (int w = 0; w < 256 / kWave; ++w)
                if (part_o[w] >= 0)
                    for (int q = 0; q < 3; ++q) {
                        gmn[q] = min(gmn[q], part[w][q]);
                        gmx[q] = max(gmx[q], part[w][3 + q]);
                    }
            for (int q = 0; q < 3; ++q) {
                atomicMin(&bounds[6 * go + q], gmn[q]);
                atomicMax(&bounds[6 * go + 3 + q], gmx[q]);
            }
        } else {
            for (int w = 0; w < 256 / kWave; ++w)
                if (part_o[w] >= 0)
                    for (int q = 0; q < 3; ++q) {
                        atomicMin(&bounds[6 * part_o[w] + q], part[w][q]);
                        atomicMax(&bounds[6 * part_o[w] + 3 + q], part[w][3 + q]);
                    }
        }
    }
}

__device__ inline uint32_t spread10(uint32_t x)
{
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// keys: Morton codes over the object's centroid bounds; vals: global triangle index
template <bool kBatch>
__global__ __launch_bounds__(256) void k_morton(Args a, const float* __restrict__ v, const int32_t* __restrict__ t,
                                                int32_t total, const uint32_t* __restrict__ bounds,
                                                uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, i);
    const float3 c = tri_centroid(v + 3 * (int64_t)s.vert_off, t + 3 * (int64_t)s.tri_off, i - s.tri_off);
    const float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        const float lo = o2f(bounds[6 * s.o + d]), hi = o2f(bounds[6 * s.o + 3 + d]);
        const float ext = hi - lo;
        float f = ext > 0.0f ? (cc[d] - lo) / ext : 0.0f;
        f = fminf(fmaxf(f * 1024.0f, 0.0f), 1023.0f);
        q[d] = (uint32_t)f;
    }
    keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[i] = (uint32_t)i;
}

// ---- segmented stable LSD radix sort, 8-bit digits ---------------------------------------
// counts[256 * tile_off + digit * ntiles + local tile] of each object
template <bool kBatch>
__global__ __launch_bounds__(kSortThreads) void k_hist(Args a, const uint32_t* __restrict__ keys, int shift,
                                                       uint32_t* __restrict__ counts)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const Seg s = seg_of_tile<kBatch>(a, blockIdx.x);
    const int32_t lt = blockIdx.x - s.tile_off;
    const int32_t first = s.tri_off + lt * kBvhSortTile, end = s.tri_off + s.nt;
    for (int r = 0; r < kSortRounds; ++r) {
        const int32_t i = first + r * kSortThreads + threadIdx.x;
        if (i < end) atomicAdd(&h[(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    counts[256 * (int64_t)s.tile_off + (int64_t)threadIdx.x * tiles_of(s.nt) + lt] = h[threadIdx.x];
}

template <bool kBatch>
__global__ __launch_bounds__(kSortThreads) void k_scatter(Args a, const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout, int shift,
                                                          const uint32_t* __restrict__ offsets)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcount[kSortThreads / kWave][256];
    const Seg s = seg_of_tile<kBatch>(a, blockIdx.x);
    const int32_t lt = blockIdx.x - s.tile_off;
    run[threadIdx.x] = offsets[256 * (int64_t)s.tile_off + (int64_t)threadIdx.x * tiles_of(s.nt) + lt];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int32_t first = s.tri_off + lt * kBvhSortTile, end = s.tri_off + s.nt;
    for (int r = 0; r < kSortRounds; ++r) {
        for (int w = 0; w < kSortThreads / kWave; ++w) wcount[w][threadIdx.x] = 0u;
        __syncthreads();
        const int32_t i = first + r * kSortThreads + threadIdx.x;
        const bool valid = i < end;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & 0xFFu;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcount[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / kWave; ++w) add += wcount[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// ---- binary nodes ----------------------------------------------------------------------
// Each stores both children's boxes, and in the spare lanes its own range of sorted
// triangles (a_hi.w = first, b_hi.w = count).  Object o's nodes are at [tri_off, tri_off
// + nt - 1) with local indices; child codes are local (>= 0 node, < 0 leaf ~position).
struct alignas(16) BinNode {
    float4 a_lo;  // xyz = child a box min, w = bits of child a
    float4 a_hi;  // xyz = child a box max, w = bits of this node's first triangle
    float4 b_lo;  // child b
    float4 b_hi;  // w = bits of this node's triangle count
};

__device__ inline int delta(const uint32_t* __restrict__ k, int32_t n, int32_t i, int32_t j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = k[i], b = k[j];
    if (a == b) return 32 + __clz((int)((uint32_t)i ^ (uint32_t)j));
    return __clz((int)(a ^ b));
}

// LBVH: Karras's radix tree; parent[] of nodes at [tri_off, ...), of leaves at lparent
template <bool kBatch>
__global__ __launch_bounds__(256) void k_tree(Args a, const uint32_t* __restrict__ keys, int32_t total,
                                              BinNode* __restrict__ bin, int32_t* __restrict__ nparent,
                                              int32_t* __restrict__ lparent)
{
    const int32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gi);
    const int32_t n = s.nt, i = gi - s.tri_off;
    if (i >= n - 1) return;
    const uint32_t* k = keys + s.tri_off;
    const int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(k, n, i, i - d);
    int32_t lmax = 2;
    while (delta(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int32_t l = 0;
    for (int32_t tt = lmax >> 1; tt >= 1; tt >>= 1)
        if (delta(k, n, i, i + (l + tt) * d) > dmin) l += tt;
    const int32_t j = i + l * d;
    const int dnode = delta(k, n, i, j);
    int32_t sp = 0;
    for (int32_t div = 2;; div <<= 1) {
        const int32_t tt = (l + div - 1) / div;
        if (delta(k, n, i, i + (sp + tt) * d) > dnode) sp += tt;
        if (tt <= 1) break;
    }
    const int32_t gamma = i + sp * d + min(d, 0);
    const int32_t left = (min(i, j) == gamma) ? ~gamma : gamma;
    const int32_t right = (max(i, j) == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    const float inf = __int_as_float(0x7f800000);
    BinNode* node = bin + s.tri_off + i;
    node->a_lo = make_float4(inf, inf, inf, __int_as_float(left));
    node->a_hi = make_float4(-inf, -inf, -inf, __int_as_float(min(i, j)));
    node->b_lo = make_float4(inf, inf, inf, __int_as_float(right));
    node->b_hi = make_float4(-inf, -inf, -inf, __int_as_float(max(i, j) - min(i, j) + 1));
    if (left >= 0) nparent[s.tri_off + left] = i;
    else lparent[s.tri_off + ~left] = i;
    if (right >= 0) nparent[s.tri_off + right] = i;
    else lparent[s.tri_off + ~right] = i;
}

template <bool kBatch>
__device__ inline BvhTri* blob_tris(char* bvh, const Seg& s)
{
    return (BvhTri*)(bvh + s.bvh_off + 256 + sizeof(Bvh4Node) * (size_t)(s.nt > 1 ? s.nt - 1 : 1));
}

template <bool kBatch>
__device__ inline BvhTri leaf_record(const float* __restrict__ v, const int32_t* __restrict__ t, const Seg& s,
                                     int32_t local_id)
{
    const float* vb = v + 3 * (int64_t)s.vert_off;
    const int32_t* tb = t + 3 * (int64_t)s.tri_off;
    const int64_t ia = tb[3 * (int64_t)local_id], ib = tb[3 * (int64_t)local_id + 1], ic = tb[3 * (int64_t)local_id + 2];
    BvhTri tri;
    tri.v0 = make_float4(vb[3 * ia], vb[3 * ia + 1], vb[3 * ia + 2], __int_as_float(local_id));
    tri.v1 = make_float4(vb[3 * ib], vb[3 * ib + 1], vb[3 * ib + 2], 0.0f);
    tri.v2 = make_float4(vb[3 * ic], vb[3 * ic + 1], vb[3 * ic + 2], 0.0f);
    return tri;
}

// ---- LBVH boxes -------------------------------------------------------------------------
// Radix-tree node i covers the consecutive sorted leaves [first, first + count) (k_tree
// stores them in its a_hi.w / b_hi.w), so its box is the union of those leaves' boxes: no
// bottom-up chain of arrivals is needed.  Level 0 of a box pyramid holds the leaf boxes
// (global sorted positions), level k + 1 the unions of kBoxFan consecutive level-k entries;
// a range query reads the partial blocks at both ends of each level and moves up through
// the whole blocks, so it reads at most 2 (kBoxFan - 1) entries per level.  A block that
// straddles two objects of a batch is never read: a node's range lies within one object and
// only blocks inside the range are used.
constexpr int kBoxFan = 64;
constexpr int kBoxLevels = 6;  // kBoxFan^5 >= kBvhMaxTris
struct LeafBox {
    float4 lo, hi;  // .w unused
};
struct BoxPyramid {
    const LeafBox* lev[kBoxLevels];
    int32_t nlev;  // levels in use; the last holds at most kBoxFan entries
};

__device__ inline void grow(float3& lo, float3& hi, const LeafBox& b)
{
    lo = make_float3(fminf(lo.x, b.lo.x), fminf(lo.y, b.lo.y), fminf(lo.z, b.lo.z));
    hi = make_float3(fmaxf(hi.x, b.hi.x), fmaxf(hi.y, b.hi.y), fmaxf(hi.z, b.hi.z));
}

// union of the level-0 entries [lo, hi] (inclusive)
__device__ inline void range_box(const BoxPyramid& P, int64_t lo, int64_t hi, float3& blo, float3& bhi)
{
    for (int k = 0; lo <= hi; ++k) {
        const LeafBox* __restrict__ c = P.lev[k];
        if (k + 1 == P.nlev) {
#pragma unroll 4
            for (int64_t e = lo; e <= hi; ++e) grow(blo, bhi, c[e]);
            break;
        }
        const int64_t head = min(hi + 1, (lo + kBoxFan - 1) / kBoxFan * kBoxFan);  // first block boundary
#pragma unroll 4
        for (int64_t e = lo; e < head; ++e) grow(blo, bhi, c[e]);
        if (head > hi) break;
        const int64_t tail = max(head, (hi + 1) / kBoxFan * kBoxFan);  // last block boundary
#pragma unroll 4
        for (int64_t e = tail; e <= hi; ++e) grow(blo, bhi, c[e]);
        lo = head / kBoxFan;
        hi = tail / kBoxFan - 1;
    }
}

// child slot of node `parent` whose code is `code`: its box components (x, y, z of lo and hi)
// are written one by one, leaving the .w fields that k_tree filled
__device__ inline void set_child_box(BinNode* node, int32_t code, float3 lo, float3 hi)
{
    const bool is_a = __float_as_int(node->a_lo.w) == code;
    float* slo = is_a ? &node->a_lo.x : &node->b_lo.x;
    float* shi = is_a ? &node->a_hi.x : &node->b_hi.x;
    slo[0] = lo.x;
    slo[1] = lo.y;
    slo[2] = lo.z;
    shi[0] = hi.x;
    shi[1] = hi.y;
    shi[2] = hi.z;
}

// LBVH leaves: the triangle records in sorted order, the leaf boxes (level 0), and each
// leaf's box in its parent's child slot
template <bool kBatch>
__global__ __launch_bounds__(256) void k_lbvh_leaves(Args a, const float* __restrict__ v,
                                                     const int32_t* __restrict__ t, int32_t total,
                                                     const uint32_t* __restrict__ order, BinNode* bin, char* bvh,
                                                     const int32_t* __restrict__ lparent, LeafBox* __restrict__ boxes)
{
    const int32_t gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gp);
    const int32_t pos = gp - s.tri_off;
    const int32_t id = (int32_t)order[gp] - s.tri_off;
    blob_tris<kBatch>(bvh, s)[pos] = leaf_record<kBatch>(v, t, s, id);
    float3 blo, bhi;
    tri_box(v + 3 * (int64_t)s.vert_off, t + 3 * (int64_t)s.tri_off, id, s.pad, blo, bhi);
    boxes[gp] = LeafBox{make_float4(blo.x, blo.y, blo.z, 0.0f), make_float4(bhi.x, bhi.y, bhi.z, 0.0f)};
    if (s.nt > 1) set_child_box(bin + s.tri_off + lparent[gp], ~pos, blo, bhi);
}

// level k + 1 of the box pyramid: one wave per block of kBoxFan level-k entries
__global__ __launch_bounds__(256) void k_box_level(const LeafBox* __restrict__ below, int64_t nbelow,
                                                   LeafBox* __restrict__ above, int64_t nabove)
{
    const int64_t blk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (blk >= nabove) return;  // whole waves leave together (nabove is a count of waves)
    const int64_t e = blk * kBoxFan + __lane_id();
    const float inf = __int_as_float(0x7f800000);
    float3 lo = make_float3(inf, inf, inf), hi = make_float3(-inf, -inf, -inf);
    if (e < nbelow) grow(lo, hi, below[e]);
    for (int m = kWave / 2; m >= 1; m >>= 1) {
        lo = make_float3(fminf(lo.x, __shfl_xor(lo.x, m)), fminf(lo.y, __shfl_xor(lo.y, m)),
                         fminf(lo.z, __shfl_xor(lo.z, m)));
        hi = make_float3(fmaxf(hi.x, __shfl_xor(hi.x, m)), fmaxf(hi.y, __shfl_xor(hi.y, m)),
                         fmaxf(hi.z, __shfl_xor(hi.z, m)));
    }
    if (__lane_id() == 0)
        above[blk] = LeafBox{make_float4(lo.x, lo.y, lo.z, 0.0f), make_float4(hi.x, hi.y, hi.z, 0.0f)};
}

// LBVH internal nodes: each node's box from its leaf range, into its parent's child slot
template <bool kBatch>
__global__ __launch_bounds__(256) void k_lbvh_nodes(Args a, int32_t total, BinNode* bin,
                                                    const int32_t* __restrict__ nparent, BoxPyramid P)
{
    const int32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gi);
    const int32_t i = gi - s.tri_off;
    if (i == 0 || i >= s.nt - 1) return;  // the root has no parent; nt - 1 internal nodes
    const BinNode* node = bin + gi;
    const int64_t first = (int64_t)s.tri_off + __float_as_int(node->a_hi.w);
    const int64_t count = __float_as_int(node->b_hi.w);
    const float inf = __int_as_float(0x7f800000);
    float3 lo = make_float3(inf, inf, inf), hi = make_float3(-inf, -inf, -inf);
    range_box(P, first, first + count - 1, lo, hi);
    set_child_box(bin + s.tri_off + nparent[gi], i, lo, hi);
}

// ---- PLOC ------------------------------------------------------------------------------
// A cluster: lo.xyz / hi.xyz its box, lo.w its code (>= 0 local node, < 0 ~global
// triangle), hi.w its object.
struct Cluster {
    float4 lo, hi;
};
static_assert(sizeof(Cluster) == sizeof(LeafBox), "the LBVH box pyramid reuses the cluster arrays");

__device__ inline float union_area(const Cluster& x, const Cluster& y)
{
    const float dx = fmaxf(x.hi.x, y.hi.x) - fminf(x.lo.x, y.lo.x);
    const float dy = fmaxf(x.hi.y, y.hi.y) - fminf(x.lo.y, y.lo.y);
    const float dz = fmaxf(x.hi.z, y.hi.z) - fminf(x.lo.z, y.lo.z);
    const float ar = dx * dy + dy * dz + dz * dx;
    return ar == ar ? ar : __int_as_float(0x7f800000);  // NaN boxes compare as +inf
}

__device__ inline Cluster merge_cluster(const Cluster& x, const Cluster& y, int32_t code)
{
    Cluster c;
    c.lo = make_float4(fminf(x.lo.x, y.lo.x), fminf(x.lo.y, y.lo.y), fminf(x.lo.z, y.lo.z), __int_as_float(code));
    c.hi = make_float4(fmaxf(x.hi.x, y.hi.x), fmaxf(x.hi.y, y.hi.y), fmaxf(x.hi.z, y.hi.z), x.hi.w);
    return c;
}

__device__ inline int32_t code_of(const Cluster& c) { return __float_as_int(c.lo.w); }
__device__ inline int32_t obj_of(const Cluster& c) { return __float_as_int(c.hi.w); }

template <bool kBatch>
__global__ __launch_bounds__(256) void k_ploc_init(Args a, const float* __restrict__ v, const int32_t* __restrict__ t,
                                                   int32_t total, const uint32_t* __restrict__ order,
                                                   Cluster* __restrict__ cl)
{
    const int32_t gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gp);
    const int32_t gt = (int32_t)order[gp];
    float3 lo, hi;
    tri_box(v + 3 * (int64_t)s.vert_off, t + 3 * (int64_t)s.tri_off, gt - s.tri_off, s.pad, lo, hi);
    cl[gp].lo = make_float4(lo.x, lo.y, lo.z, __int_as_float(~gt));
    cl[gp].hi = make_float4(hi.x, hi.y, hi.z, __int_as_float(s.o));
}

// nearest neighbour of each cluster among the same object's clusters within +-kPlocRadius
// positions: least (merged area, position); -1 when the object has no other cluster there
__device__ inline int32_t nearest(const Cluster* c, int32_t i, int32_t lo, int32_t hi, int32_t base)
{
    // c: clusters indexed from `base`; candidates j in [lo, hi] (global positions)
    const Cluster me = c[i - base];
    const int32_t mo = obj_of(me);
    float best = __int_as_float(0x7f800000);
    int32_t bj = -1;
    for (int32_t j = lo; j <= hi; ++j) {
        if (j == i) continue;
        const Cluster o = c[j - base];
        if (obj_of(o) != mo) continue;
        const float ar = union_area(me, o);
        if (bj < 0 || ar < best) {
            best = ar;
            bj = j;
        }
    }
    return bj;
}

__global__ __launch_bounds__(kPlocThreads) void k_ploc_nn(const Cluster* __restrict__ cl, const int32_t* __restrict__ cseg,
                                                          int32_t nobj, int32_t* __restrict__ nn)
{
    __shared__ Cluster tile[kPlocThreads + 2 * kPlocRadius];
    const int32_t n = cseg[nobj];
    const int32_t b0 = blockIdx.x * kPlocThreads;
    if (b0 >= n) return;
    const int32_t lo = max(b0 - kPlocRadius, 0), hi = min(b0 + kPlocThreads + kPlocRadius, n);
    for (int32_t j = lo + (int32_t)threadIdx.x; j < hi; j += kPlocThreads) tile[j - lo] = cl[j];
    __syncthreads();
    const int32_t i = b0 + threadIdx.x;
    if (i >= n) return;
    nn[i] = nearest(tile, i, max(i - kPlocRadius, 0), min(i + kPlocRadius, n - 1), lo);
}

// flags[i] = merged << 32 | kept (for the exclusive scan that follows); zero past the end
__global__ void k_ploc_flags(const int32_t* __restrict__ nn, const int32_t* __restrict__ cseg, int32_t nobj,
                             int64_t cap, uint64_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > cap) return;
    const int32_t n = cseg[nobj];
    uint64_t f = 0;
    if (i < n) {
        const int32_t j = nn[i];
        const bool mutual = j >= 0 && nn[j] == (int32_t)i;
        f = ((uint64_t)(mutual && i < j) << 32) | (uint64_t)(!mutual || i < j);
    }
    flags[i] = f;
}

// per object: its first merge rank this iteration, its merge count so far, its new start
__global__ void k_ploc_seg(const int32_t* __restrict__ cseg_in, int32_t* __restrict__ cseg_out, int32_t nobj,
                           const uint64_t* __restrict__ flags, int32_t* __restrict__ base, int32_t* __restrict__ mrank0,
                           int32_t* __restrict__ mbase)
{
    const int32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o > nobj) return;
    const uint64_t fs = flags[cseg_in[o]];
    cseg_out[o] = (int32_t)(uint32_t)fs;
    if (o == nobj) return;
    const uint64_t fe = flags[cseg_in[o + 1]];
    const int32_t r0 = (int32_t)(fs >> 32), m = (int32_t)(fe >> 32) - r0;
    mrank0[o] = r0;
    mbase[o] = base[o];
    base[o] += m;
}

// writes merged node `id` of object `s` from clusters x (left) and y (right)
template <bool kBatch>
__device__ inline void write_node(const Seg& s, int32_t id, const Cluster& x, const Cluster& y, BinNode* __restrict__ bin,
                                  int32_t* __restrict__ ncount, int32_t* __restrict__ nparent,
                                  int32_t* __restrict__ lparent)
{
    const int32_t cx = code_of(x), cy = code_of(y);
    BinNode nd;
    nd.a_lo = x.lo;
    nd.a_hi = make_float4(x.hi.x, x.hi.y, x.hi.z, 0.0f);
    nd.b_lo = y.lo;
    nd.b_hi = make_float4(y.hi.x, y.hi.y, y.hi.z, 0.0f);
    bin[s.tri_off + id] = nd;
    const int32_t nx = cx >= 0 ? ncount[s.tri_off + cx] : 1, ny = cy >= 0 ? ncount[s.tri_off + cy] : 1;
    ncount[s.tri_off + id] = nx + ny;
    if (cx >= 0) nparent[s.tri_off + cx] = id;
    else lparent[~cx] = id;
    if (cy >= 0) nparent[s.tri_off + cy] = id;
    else lparent[~cy] = id;
}

template <bool kBatch>
__global__ __launch_bounds__(256) void k_ploc_compact(Args a, const Cluster* __restrict__ cin, Cluster* __restrict__ cout,
                                                      const int32_t* __restrict__ cseg_in, int32_t nobj,
                                                      const int32_t* __restrict__ nn, const uint64_t* __restrict__ flags,
                                                      const int32_t* __restrict__ mrank0, const int32_t* __restrict__ mbase,
                                                      BinNode* __restrict__ bin, int32_t* __restrict__ ncount,
                                                      int32_t* __restrict__ nparent, int32_t* __restrict__ lparent)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cseg_in[nobj]) return;
    const uint64_t f = flags[i], f1 = flags[i + 1];
    const uint32_t keep = (uint32_t)f1 - (uint32_t)f, merged = (uint32_t)(f1 >> 32) - (uint32_t)(f >> 32);
    if (!keep) return;
    const uint32_t pos = (uint32_t)f;
    const Cluster me = cin[i];
    if (!merged) {
        cout[pos] = me;
        return;
    }
    const int32_t j = nn[i];
    const Cluster other = cin[j];
    const int32_t o = obj_of(me);
    const Seg s = seg_of_obj<kBatch>(a, o);
    const int32_t id = s.nt - 2 - (mbase[o] + ((int32_t)(f >> 32) - mrank0[o]));
    write_node<kBatch>(s, id, me, other, bin, ncount, nparent, lparent);
    cout[pos] = merge_cluster(me, other, id);
}

// Exclusive scans of keep and mrg over a work-group of kFinishThreads (one value per
// thread); returns this thread's prefixes and writes the totals into tot.
__device__ inline void finish_scan(uint32_t keep, uint32_t mrg, uint32_t* s_keep, uint32_t* s_merge, uint32_t& pk,
                                   uint32_t& pm, uint32_t& tk, uint32_t& tm)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    uint32_t ik = keep, im = mrg;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t xk = __shfl_up(ik, d, kWave), xm = __shfl_up(im, d, kWave);
        if (lane >= d) {
            ik += xk;
            im += xm;
        }
    }
    if (lane == kWave - 1) {
        s_keep[wave] = ik;
        s_merge[wave] = im;
    }
    __syncthreads();
    pk = ik - keep;
    pm = im - mrg;
    tk = 0;
    tm = 0;
    for (int w = 0; w < kFinishThreads / kWave; ++w) {
        if (w < wave) {
            pk += s_keep[w];
            pm += s_merge[w];
        }
        tk += s_keep[w];
        tm += s_merge[w];
    }
    __syncthreads();  // s_keep / s_merge are reused by the next scan
}

// One work-group per object finishes its clusters [start, start + n) of buffer A, using
// the same segment of buffer B as the other half of the ping-pong, `nnw` for the nearest
// neighbours and LDS scans for the compaction; once at most kFinishLds clusters remain they
// move to LDS and the remaining iterations run there (every read of an iteration happens
// before a barrier, every write after it, so the compaction is in place).  Every iteration
// merges at least one pair (the least (area, position) pair of the object is mutual), so it
// ends after at most n - 1 iterations.
constexpr int32_t kFinishLds = 1792;  // 56 KB of clusters + 7 KB of neighbour indices
static_assert(kFinishLds <= 2 * kFinishThreads, "two clusters per thread in the LDS phase");

template <bool kBatch>
__global__ __launch_bounds__(kFinishThreads) void k_ploc_finish(Args a, Cluster* ca, Cluster* cb,
                                                                const int32_t* __restrict__ cseg, const int32_t* base_in,
                                                                int32_t* nnw, BinNode* __restrict__ bin,
                                                                int32_t* __restrict__ ncount, int32_t* __restrict__ nparent,
                                                                int32_t* __restrict__ lparent)
{
    __shared__ uint32_t s_keep[kFinishThreads / kWave], s_merge[kFinishThreads / kWave];
    __shared__ uint32_t s_tot[2];
    __shared__ Cluster s_cl[kFinishLds];
    __shared__ int32_t s_nn[kFinishLds];
    const int32_t o = blockIdx.x;
    const Seg s = seg_of_obj<kBatch>(a, o);
    const int32_t start = cseg[o];
    int32_t n = cseg[o + 1] - start;
    int32_t merges = base_in[o];
    Cluster* cur = ca;
    Cluster* nxt = cb;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int32_t guard = 0;
    for (; n > kFinishLds && guard < s.nt; ++guard) {
        for (int32_t i = tid; i < n; i += kFinishThreads)
            nnw[start + i] = nearest(cur + start, i, max(i - kPlocRadius, 0), min(i + kPlocRadius, n - 1), 0);
        __syncthreads();
        uint32_t kept_total = 0, merged_total = 0;
        for (int32_t c0 = 0; c0 < n; c0 += kFinishThreads) {
            const int32_t i = c0 + tid;
            uint32_t keep = 0, mrg = 0;
            int32_t j = -1;
            if (i < n) {
                j = nnw[start + i];
                const bool mutual = j >= 0 && nnw[start + j] == i;
                keep = (!mutual || i < j) ? 1u : 0u;
                mrg = (mutual && i < j) ? 1u : 0u;
            }
            // exclusive scans of keep and mrg over the work-group
            uint32_t ik = keep, im = mrg;
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t xk = __shfl_up(ik, d, kWave), xm = __shfl_up(im, d, kWave);
                if (lane >= d) {
                    ik += xk;
                    im += xm;
                }
            }
            if (lane == kWave - 1) {
                s_keep[wave] = ik;
                s_merge[wave] = im;
            }
            __syncthreads();
            uint32_t pk = kept_total + ik - keep, pm = merged_total + im - mrg;
            for (int w = 0; w < wave; ++w) {
                pk += s_keep[w];
                pm += s_merge[w];
            }
            if (tid == kFinishThreads - 1) {
                s_tot[0] = pk + keep;
                s_tot[1] = pm + mrg;
            }
            if (keep) {
                const Cluster me = cur[start + i];
                if (mrg) {
                    const Cluster other = cur[start + j];
                    const int32_t id = s.nt - 2 - (merges + (int32_t)pm);
                    write_node<kBatch>(s, id, me, other, bin, ncount, nparent, lparent);
                    nxt[start + pk] = merge_cluster(me, other, id);
                } else {
                    nxt[start + pk] = me;
                }
            }
            __syncthreads();
            kept_total = s_tot[0];
            merged_total = s_tot[1];
        }
        merges += (int32_t)merged_total;
        n = (int32_t)kept_total;
        Cluster* tmp = cur;
        cur = nxt;
        nxt = tmp;
        __syncthreads();
    }
    if (n <= 1) return;
    // LDS phase: at most kFinishLds clusters, two per thread
    for (int32_t i = tid; i < n; i += kFinishThreads) s_cl[i] = cur[start + i];
    __syncthreads();
    for (; n > 1 && guard < s.nt; ++guard) {
        for (int32_t i = tid; i < n; i += kFinishThreads)
            s_nn[i] = nearest(s_cl, i, max(i - kPlocRadius, 0), min(i + kPlocRadius, n - 1), 0);
        __syncthreads();
        Cluster me[2], other[2];
        uint32_t keep[2] = {0u, 0u}, mrg[2] = {0u, 0u};
        for (int r = 0; r < 2; ++r) {
            const int32_t i = r * kFinishThreads + tid;
            if (i < n) {
                const int32_t j = s_nn[i];
                const bool mutual = j >= 0 && s_nn[j] == i;
                keep[r] = (!mutual || i < j) ? 1u : 0u;
                mrg[r] = (mutual && i < j) ? 1u : 0u;
                me[r] = s_cl[i];
                if (mrg[r]) other[r] = s_cl[j];
            }
        }
        uint32_t pk0, pm0, tk0, tm0, pk1, pm1, tk1, tm1;
        finish_scan(keep[0], mrg[0], s_keep, s_merge, pk0, pm0, tk0, tm0);  // its barriers end the reads
        finish_scan(keep[1], mrg[1], s_keep, s_merge, pk1, pm1, tk1, tm1);
        const uint32_t pk[2] = {pk0, tk0 + pk1}, pm[2] = {pm0, tm0 + pm1};
        for (int r = 0; r < 2; ++r) {
            if (!keep[r]) continue;
            if (mrg[r]) {
                const int32_t id = s.nt - 2 - (merges + (int32_t)pm[r]);
                write_node<kBatch>(s, id, me[r], other[r], bin, ncount, nparent, lparent);
                s_cl[pk[r]] = merge_cluster(me[r], other[r], id);
            } else {
                s_cl[pk[r]] = me[r];
            }
        }
        __syncthreads();
        merges += (int32_t)(tm0 + tm1);
        n = (int32_t)(tk0 + tk1);
    }
}

// PLOC: every leaf walks to the root for its depth-first position; writes its record
template <bool kBatch>
__global__ __launch_bounds__(256) void k_ploc_leaves(Args a, const float* __restrict__ v, const int32_t* __restrict__ t,
                                                     int32_t total, const BinNode* __restrict__ bin,
                                                     const int32_t* __restrict__ ncount, const int32_t* __restrict__ nparent,
                                                     const int32_t* __restrict__ lparent, int32_t* __restrict__ posmap,
                                                     char* bvh)
{
    const int32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    if (gt >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gt);
    int32_t pos = 0, me = ~gt, p = lparent[gt];
    for (int32_t guard = 0; p >= 0 && guard < s.nt; ++guard) {
        const BinNode& nd = bin[s.tri_off + p];
        if (__float_as_int(nd.b_lo.w) == me) {
            const int32_t ca = __float_as_int(nd.a_lo.w);
            pos += ca >= 0 ? ncount[s.tri_off + ca] : 1;
        }
        me = p;
        p = nparent[s.tri_off + p];
    }
    posmap[gt] = pos;
    blob_tris<kBatch>(bvh, s)[pos] = leaf_record<kBatch>(v, t, s, gt - s.tri_off);
}

// PLOC: node ranges (first by the same walk) and leaf codes as positions
template <bool kBatch>
__global__ __launch_bounds__(256) void k_ploc_nodes(Args a, int32_t total, BinNode* __restrict__ bin,
                                                    const int32_t* __restrict__ ncount,
                                                    const int32_t* __restrict__ nparent,
                                                    const int32_t* __restrict__ posmap)
{
    const int32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= total) return;
    const Seg s = seg_of_tri<kBatch>(a, gi);
    const int32_t id = gi - s.tri_off;
    if (id >= s.nt - 1) return;
    int32_t first = 0, me = id, p = nparent[gi];
    for (int32_t guard = 0; p >= 0 && guard < s.nt; ++guard) {
        const BinNode& nd = bin[s.tri_off + p];
        if (__float_as_int(nd.b_lo.w) == me) {
            const int32_t ca = __float_as_int(nd.a_lo.w);
            first += ca >= 0 ? ncount[s.tri_off + ca] : 1;
        }
        me = p;
        p = nparent[s.tri_off + p];
    }
    BinNode& nd = bin[gi];
    const int32_t ca = __float_as_int(nd.a_lo.w), cb = __float_as_int(nd.b_lo.w);
    nd.a_lo.w = __int_as_float(ca >= 0 ? ca : ~posmap[~ca]);
    nd.b_lo.w = __int_as_float(cb >= 0 ? cb : ~posmap[~cb]);
    nd.a_hi.w = __int_as_float(first);
    nd.b_hi.w = __int_as_float(ncount[gi]);
}

// ---- collapse into a 4-wide hierarchy ---------------------------------------------------
// For every binary node: start from its two children and repeatedly open the child with
// the largest surface area that holds more than kLeafMax triangles, until there are 4
// children or nothing left to open; children with at most kLeafMax triangles become leaf
// ranges (every subtree covers consecutive triangles).  Each node's result depends only on
// its own subtree, so all nodes are collapsed in parallel; the ones reachable from the
// root form the hierarchy.
struct Slot {
    int32_t code;   // binary code: >= 0 node, < 0 leaf ~position
    int32_t first, count;
    float3 lo, hi;
};

__device__ inline Slot child_slot(const BinNode* __restrict__ nodes, const BinNode& par, bool a)
{
    Slot s;
    const float4 lo = a ? par.a_lo : par.b_lo, hi = a ? par.a_hi : par.b_hi;
    s.code = __float_as_int(lo.w);
    s.lo = make_float3(lo.x, lo.y, lo.z);
    s.hi = make_float3(hi.x, hi.y, hi.z);
    if (s.code >= 0) {
        s.first = __float_as_int(nodes[s.code].a_hi.w);
        s.count = __float_as_int(nodes[s.code].b_hi.w);
    } else {
        s.first = ~s.code;
        s.count = 1;
    }
    return s;
}

__device__ inline float half_area(const Slot& s)
{
    const float dx = s.hi.x - s.lo.x, dy = s.hi.y - s.lo.y, dz = s.hi.z - s.lo.z;
    return dx * dy + dy * dz + dz * dx;
}

template <bool kBatch>
__global__ __launch_bounds__(256) void k_collapse4(Args a, const BinNode* __restrict__ bin, int32_t total, char* bvh)
{
    const int32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= total) return;
    const Seg sg = seg_of_tri<kBatch>(a, gi);
    const int32_t i = gi - sg.tri_off;
    if (i >= sg.nt - 1) return;
    const BinNode* nodes = bin + sg.tri_off;
    Slot s[4];
    const BinNode me = nodes[i];
    s[0] = child_slot(nodes, me, true);
    s[1] = child_slot(nodes, me, false);
    int m = 2;
    while (m < 4) {
        int best = -1;
        float area = -1.0f;
        for (int q = 0; q < m; ++q)
            if (s[q].code >= 0 && s[q].count > kLeafMax && half_area(s[q]) > area) {
                area = half_area(s[q]);
                best = q;
            }
        if (best < 0) break;
        const BinNode c = nodes[s[best].code];
        s[m] = child_slot(nodes, c, false);
        s[best] = child_slot(nodes, c, true);
        ++m;
    }
    // the node box (the children's union) and, per axis, the least power-of-two step s with
    // 255 s >= the box's extent; planes are quantised in binary64, where the differences of
    // binary32 coordinates and the division by s are exact for coordinates of comparable
    // magnitude (any rounding elsewhere stays far below the boxes' 2 * pad widening)
    float3 blo = s[0].lo, bhi = s[0].hi;
    for (int q = 1; q < m; ++q) {
        blo = make_float3(fminf(blo.x, s[q].lo.x), fminf(blo.y, s[q].lo.y), fminf(blo.z, s[q].lo.z));
        bhi = make_float3(fmaxf(bhi.x, s[q].hi.x), fmaxf(bhi.y, s[q].hi.y), fmaxf(bhi.z, s[q].hi.z));
    }
    const float bl[3] = {blo.x, blo.y, blo.z}, bh[3] = {bhi.x, bhi.y, bhi.z};
    Bvh4Node o;
    o.ox = blo.x;
    o.oy = blo.y;
    o.oz = blo.z;
    o.exps = 0u;
    for (int ax = 0; ax < 3; ++ax) {
        const double ext = (double)bh[ax] - (double)bl[ax];
        int k = -126;
        if (ext > 0.0) {
            int p;
            frexp(ext / 255.0, &p);   // ext / 255 < 2^p
            k = max(p, -126);
        }
        const double step = ldexp(1.0, k);
        o.exps |= (uint32_t)(k + 127) << (8 * ax);
        uint32_t lw = 0u, hw = 0u;
        for (int q = 0; q < 4; ++q) {
            uint32_t ql = 255u, qh = 0u;  // unused slot: an inverted box
            if (q < m) {
                const float cl = ax == 0 ? s[q].lo.x : (ax == 1 ? s[q].lo.y : s[q].lo.z);
                const float ch = ax == 0 ? s[q].hi.x : (ax == 1 ? s[q].hi.y : s[q].hi.z);
                ql = (uint32_t)min(max(floor(((double)cl - (double)bl[ax]) / step), 0.0), 255.0);
                qh = (uint32_t)min(max(ceil(((double)ch - (double)bl[ax]) / step), 0.0), 255.0);
            }
            lw |= ql << (8 * q);
            hw |= qh << (8 * q);
        }
        o.lo[ax] = lw;
        o.hi[ax] = hw;
    }
    int32_t cc[4];
    for (int q = 0; q < 4; ++q)
        cc[q] = q >= m ? kBvhEmptySlot : (s[q].count <= kLeafMax ? leaf_code(s[q].first, s[q].count) : s[q].code);
    o.child = make_int4(cc[0], cc[1], cc[2], cc[3]);
    o.unused[0] = o.unused[1] = 0u;
    ((Bvh4Node*)(bvh + sg.bvh_off + 256))[i] = o;
}

// The 4-wide depth (nodes on the longest root-to-leaf path) of the collapsed hierarchy.
// Every binary subtree covers consecutive triangle positions (its first and count are in
// its node), so each triangle walks down from the root, entering at each 4-wide node the
// child node whose range holds its position, until a leaf range holds it; the deepest walk
// is the depth, which goes into the header with one atomicMax per object and work-group
// (the header's depth starts at 0; a root that is a leaf range keeps it).
template <bool kBatch>
__global__ __launch_bounds__(256) void k_depth4(Args a, const BinNode* __restrict__ bin, int32_t total, char* bvh)
{
    const int32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gt < total;  // lanes past the end stay for the reductions below
    int32_t depth = 0;
    int32_t* slot = nullptr;
    if (live) {
        const Seg s = seg_of_tri<kBatch>(a, gt);
        slot = &((BvhHeader*)(bvh + s.bvh_off))->depth;
        if (s.nt > kLeafMax) {
            const Bvh4Node* n4 = (const Bvh4Node*)(bvh + s.bvh_off + 256);
            const BinNode* nodes = bin + s.tri_off;
            const uint32_t pos = (uint32_t)(gt - s.tri_off);
            int32_t p = 0;
            depth = 1;
            for (int32_t guard = 0; guard < s.nt; ++guard) {
                const int4 c = n4[p].child;
                const int32_t cc[4] = {c.x, c.y, c.z, c.w};
                int32_t next = -1;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (cc[q] >= 0) {
                        const uint32_t first = (uint32_t)__float_as_int(nodes[cc[q]].a_hi.w);
                        const uint32_t count = (uint32_t)__float_as_int(nodes[cc[q]].b_hi.w);
                        if (pos - first < count) next = cc[q];
                    }
                if (next < 0) break;
                p = next;
                ++depth;
            }
        }
    }
    // one atomic per work-group when its live triangles belong to one object (atomics on one
    // address serialise across the chip), else one per wave or lane
    __shared__ int32_t* wslot[256 / kWave];
    __shared__ int32_t wdepth[256 / kWave];
    const int wave = threadIdx.x / kWave;
    const uint64_t lives = __ballot(live);
    int32_t* ws = nullptr;
    int32_t m = depth;  // 0 on the lanes past the end
    if (lives != 0ull) {
        const int32_t first_lane = __ffsll((long long)lives) - 1;
        const uintptr_t obj0 = (uintptr_t)__shfl((int64_t)(uintptr_t)slot, first_lane);
        if (__ballot(live && (uintptr_t)slot != obj0) == 0ull) {
            for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d));
            ws = (int32_t*)obj0;
        } else if (live) {
            atomicMax(slot, depth);
        }
    }
    if (__lane_id() == 0) {
        wslot[wave] = ws;
        wdepth[wave] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t* gs = nullptr;
        bool one = true;
        int32_t gm = 0;
        for (int w = 0; w < 256 / kWave; ++w) {
            if (wslot[w] == nullptr) continue;
            if (gs == nullptr) gs = wslot[w];
            else if (wslot[w] != gs) one = false;
            gm = max(gm, wdepth[w]);
        }
        if (gs != nullptr && one) {
            atomicMax(gs, gm);
        } else {
            for (int w = 0; w < 256 / kWave; ++w)
                if (wslot[w] != nullptr) atomicMax(wslot[w], wdepth[w]);
        }
    }
}

// the header (its reserved words zero) and, when no binary node exists (nt <= 1), the
// unused node slot, so that every byte of a blob is defined
template <bool kBatch>
__global__ void k_header(Args a, char* bvh)
{
    const int32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (kBatch ? a.nobj : 1)) return;
    const Seg s = seg_of_obj<kBatch>(a, o);
    int4* raw = (int4*)(bvh + s.bvh_off);
    const int words = (int)(sizeof(BvhHeader) + (s.nt <= 1 ? sizeof(Bvh4Node) : 0)) / 16;
    for (int q = 0; q < words; ++q) raw[q] = make_int4(0, 0, 0, 0);
    BvhHeader* h = (BvhHeader*)(bvh + s.bvh_off);
    h->nt = s.nt;
    h->root = s.nt <= kLeafMax ? (s.nt > 0 ? leaf_code(0, s.nt) : kBvhEmptySlot) : 0;
    h->pad = s.pad;
}

// ---- workspace ----------------------------------------------------------------------------
struct Work {
    uint32_t *k0, *v0, *k1, *v1, *counts, *bounds;
    Cluster *ca, *cb;
    int32_t *nn, *ncount, *nparent, *lparent, *posmap, *cseg0, *cseg1, *base, *mrank0, *mbase;
    uint64_t* flags;
    BinNode* bin;
    void* scan;
};

Work carve(void* work, int64_t n, int64_t tiles, int32_t nobj)
{
    Work w;
    char* p = (char*)work;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += align256(bytes);
        return (void*)r;
    };
    w.k0 = (uint32_t*)take(4 * n);
    w.v0 = (uint32_t*)take(4 * n);
    w.k1 = (uint32_t*)take(4 * n);
    w.v1 = (uint32_t*)take(4 * n);
    w.counts = (uint32_t*)take(4 * 256 * tiles);
    w.bounds = (uint32_t*)take(4 * 6 * (size_t)nobj);
    w.ca = (Cluster*)take(sizeof(Cluster) * n);
    w.cb = (Cluster*)take(sizeof(Cluster) * n);
    w.nn = (int32_t*)take(4 * n);
    w.ncount = (int32_t*)take(4 * n);
    w.nparent = (int32_t*)take(4 * n);
    w.lparent = (int32_t*)take(4 * n);
    w.posmap = (int32_t*)take(4 * n);
    w.cseg0 = (int32_t*)take(4 * ((size_t)nobj + 1));
    w.cseg1 = (int32_t*)take(4 * ((size_t)nobj + 1));
    w.base = (int32_t*)take(4 * (size_t)nobj);
    w.mrank0 = (int32_t*)take(4 * (size_t)nobj);
    w.mbase = (int32_t*)take(4 * (size_t)nobj);
    w.flags = (uint64_t*)take(8 * (n + 1));
    w.bin = (BinNode*)take(sizeof(BinNode) * n);
    w.scan = p;
    return w;
}

size_t carve_bytes(int64_t n, int64_t tiles, int32_t nobj)
{
    const size_t head = 4 * align256(4 * n) + align256(4 * 256 * tiles) + align256(4 * 6 * (size_t)nobj) +
                        2 * align256(sizeof(Cluster) * n) + 5 * align256(4 * n) +
                        2 * align256(4 * ((size_t)nobj + 1)) + 3 * align256(4 * (size_t)nobj) + align256(8 * (n + 1)) +
                        align256(sizeof(BinNode) * n);
    return head + std::max(scan_work_bytes_u32(256 * tiles), scan_work_bytes_u64(n + 1));
}

template <bool kBatch>
hipError_t build(Args a, int32_t nobj, int64_t n, int64_t tiles, const float* verts, const int32_t* tris, char* bvh,
                 void* work, int32_t method, hipStream_t s)
{
    const unsigned ob = (unsigned)ceil_div(nobj + 1, 256);
    hipLaunchKernelGGL(k_header<kBatch>, dim3(ob), dim3(256), 0, s, a, bvh);
    if (n == 0) return hipGetLastError();
    Work w = carve(work, n, tiles, nobj);
    const unsigned tb = (unsigned)ceil_div(n, 256);
    const int32_t total = (int32_t)n;
    hipLaunchKernelGGL(k_init<kBatch>, dim3(ob), dim3(256), 0, s, a, w.bounds, w.cseg0, w.base, n);
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min<unsigned>(tb, 2048u)), dim3(256), 0, s, w.nparent, n, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min<unsigned>(tb, 2048u)), dim3(256), 0, s, w.lparent, n, -1);
    hipLaunchKernelGGL(k_bounds<kBatch>, dim3((unsigned)ceil_div(total, 256 * kBoundsItems)), dim3(256), 0, s, a, verts,
                       tris, total, w.bounds);
    hipLaunchKernelGGL(k_morton<kBatch>, dim3(tb), dim3(256), 0, s, a, verts, tris, total, (const uint32_t*)w.bounds,
                       w.k0, w.v0);
    uint32_t *ka = w.k0, *va = w.v0, *kb = w.k1, *vb = w.v1;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_hist<kBatch>, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, a, ka, shift, w.counts);
        hipError_t e = scan_exclusive_u32(w.counts, w.counts, 256 * tiles, nullptr, w.scan, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scatter<kBatch>, dim3((unsigned)tiles), dim3(kSortThreads), 0, s, a, ka, va, kb, vb, shift,
                           (const uint32_t*)w.counts);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (method == RTSDF_BVH_LBVH) {
        // the radix tree, then its boxes from a box pyramid over the sorted leaves (the PLOC
        // cluster arrays hold the pyramid: level 0 in ca, the upper levels in cb)
        hipLaunchKernelGGL(k_tree<kBatch>, dim3(tb), dim3(256), 0, s, a, ka, total, w.bin, w.nparent, w.lparent);
        BoxPyramid P{};
        P.lev[0] = (const LeafBox*)w.ca;
        P.nlev = 1;
        hipLaunchKernelGGL(k_lbvh_leaves<kBatch>, dim3(tb), dim3(256), 0, s, a, verts, tris, total, va, w.bin, bvh,
                           w.lparent, (LeafBox*)w.ca);
        LeafBox* up = (LeafBox*)w.cb;  // levels 1.. take ceil(n/64) + ceil(n/64^2) + ... <= n entries
        for (int64_t cnt = n; cnt > kBoxFan && P.nlev < kBoxLevels; ++P.nlev) {
            const int64_t nup = ceil_div(cnt, kBoxFan);
            hipLaunchKernelGGL(k_box_level, dim3((unsigned)ceil_div(nup * kWave, 256)), dim3(256), 0, s,
                               P.lev[P.nlev - 1], cnt, up, nup);
            P.lev[P.nlev] = up;
            up += nup;
            cnt = nup;
        }
        hipLaunchKernelGGL(k_lbvh_nodes<kBatch>, dim3(tb), dim3(256), 0, s, a, total, w.bin, w.nparent, P);
    } else {
        hipLaunchKernelGGL(k_ploc_init<kBatch>, dim3(tb), dim3(256), 0, s, a, verts, tris, total, va, w.ca);
        Cluster *cin = w.ca, *cout = w.cb;
        int32_t *sin = w.cseg0, *sout = w.cseg1;
        const unsigned nb = (unsigned)ceil_div(n, kPlocThreads), fb = (unsigned)ceil_div(n + 1, 256);
        for (int it = 0; it < kPlocWide; ++it) {
            hipLaunchKernelGGL(k_ploc_nn, dim3(nb), dim3(kPlocThreads), 0, s, cin, sin, nobj, w.nn);
            hipLaunchKernelGGL(k_ploc_flags, dim3(fb), dim3(256), 0, s, w.nn, sin, nobj, n, w.flags);
            hipError_t e = scan_exclusive_u64(w.flags, w.flags, n + 1, nullptr, w.scan, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_ploc_seg, dim3(ob), dim3(256), 0, s, sin, sout, nobj, w.flags, w.base, w.mrank0,
                               w.mbase);
            hipLaunchKernelGGL(k_ploc_compact<kBatch>, dim3(tb), dim3(256), 0, s, a, cin, cout, sin, nobj, w.nn,
                               w.flags, w.mrank0, w.mbase, w.bin, w.ncount, w.nparent, w.lparent);
            std::swap(cin, cout);
            std::swap(sin, sout);
        }
        hipLaunchKernelGGL(k_ploc_finish<kBatch>, dim3((unsigned)nobj), dim3(kFinishThreads), 0, s, a, cin, cout, sin,
                           w.base, w.nn, w.bin, w.ncount, w.nparent, w.lparent);
        hipLaunchKernelGGL(k_ploc_leaves<kBatch>, dim3(tb), dim3(256), 0, s, a, verts, tris, total, w.bin, w.ncount,
                           w.nparent, w.lparent, w.posmap, bvh);
        hipLaunchKernelGGL(k_ploc_nodes<kBatch>, dim3(tb), dim3(256), 0, s, a, total, w.bin, w.ncount, w.nparent,
                           w.posmap);
    }
    hipLaunchKernelGGL(k_collapse4<kBatch>, dim3(tb), dim3(256), 0, s, a, (const BinNode*)w.bin, total, bvh);
    hipLaunchKernelGGL(k_depth4<kBatch>, dim3(tb), dim3(256), 0, s, a, (const BinNode*)w.bin, total, bvh);
    return hipGetLastError();
}

}  // namespace

size_t bvh_bytes(int32_t nt)
{
    return 256 + sizeof(Bvh4Node) * bvh_node_count(nt) + sizeof(BvhTri) * (size_t)nt;
}

size_t bvh_work_bytes(int64_t total_tris, int64_t total_tiles, int32_t nobj)
{
    return carve_bytes(std::max<int64_t>(total_tris, 1), std::max<int64_t>(total_tiles, 1), nobj);
}

hipError_t build_bvh(const float* verts, const int32_t* tris, int32_t nt, const rtsdf_grid& g, void* bvh, void* work,
                     int32_t method, hipStream_t s)
{
    Args a{nullptr, 1, nt, g.h * (1.0f / 256.0f)};
    return build<false>(a, 1, nt, ceil_div(nt, kBvhSortTile), verts, tris, (char*)bvh, work, method, s);
}

hipError_t build_bvh_batched(const BatchView& hv, const void* dplan, const float* verts, const int32_t* tris,
                             void* bvh, void* work, int32_t method, hipStream_t s)
{
    Args a{(const char*)dplan, hv.h->nobj, 0, 0.0f};
    return build<true>(a, hv.h->nobj, hv.h->total_tris, hv.h->total_tiles, verts, tris, (char*)bvh, work, method, s);
}

}  // namespace rtsdf
