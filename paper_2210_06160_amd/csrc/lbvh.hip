// Software linear BVH for the ray sampling of section 2.1 (the paper relies on the
// graphics driver's hierarchy and RT cores; gfx950 has neither).
//
//   centroid bounds (atomic min/max on order-preserving float encodings)
//   -> 30-bit Morton code per triangle centroid
//   -> stable LSD radix sort of (code, triangle) in four 8-bit passes
//   -> binary radix tree over the sorted codes (Karras 2012, "Maximizing parallelism in
//      the construction of BVHs, octrees, and k-d trees"); equal codes are ordered by
//      position, so every key is unique
//   -> bottom-up refit: each leaf walks to the root; the second child to arrive at a
//      node merges both boxes.
// Each internal node stores both children's boxes so that traversal tests two children
// with one 64-byte fetch.  Boxes are widened so traversal is exact (see raysample.hip).
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 4;
constexpr int kSortTile = kSortThreads * kSortRounds;

__device__ inline uint32_t f2o(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float o2f(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ inline float3 tri_centroid(const float* __restrict__ v, const int32_t* __restrict__ t,
                                      int32_t i)
{
    const int64_t a = t[3 * (int64_t)i], b = t[3 * (int64_t)i + 1], c = t[3 * (int64_t)i + 2];
    const float third = 1.0f / 3.0f;
    return make_float3((v[3 * a] + v[3 * b] + v[3 * c]) * third,
                       (v[3 * a + 1] + v[3 * b + 1] + v[3 * c + 1]) * third,
                       (v[3 * a + 2] + v[3 * b + 2] + v[3 * c + 2]) * third);
}

__global__ void k_init(uint32_t* __restrict__ bounds, uint32_t* __restrict__ flags, int32_t nflags)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 3) bounds[i] = 0xFFFFFFFFu;         // running min (encoded)
    else if (i < 6) bounds[i] = 0u;             // running max (encoded)
    for (int32_t f = i; f < nflags; f += gridDim.x * blockDim.x) flags[f] = 0u;
}

__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ v,
                                                const int32_t* __restrict__ t, int32_t nt,
                                                uint32_t* __restrict__ bounds)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
    if (i < nt) {
        const float3 c = tri_centroid(v, t, i);
        mn[0] = mx[0] = f2o(c.x);
        mn[1] = mx[1] = f2o(c.y);
        mn[2] = mx[2] = f2o(c.z);
    }
    for (int d = kWave / 2; d > 0; d >>= 1)
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], d, kWave));
            mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], d, kWave));
        }
    if ((threadIdx.x & (kWave - 1)) == 0)
        for (int a = 0; a < 3; ++a) {
            atomicMin(&bounds[a], mn[a]);
            atomicMax(&bounds[3 + a], mx[a]);
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

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ v,
                                                const int32_t* __restrict__ t, int32_t nt,
                                                const uint32_t* __restrict__ bounds,
                                                uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const float3 c = tri_centroid(v, t, i);
    const float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const float lo = o2f(bounds[a]), hi = o2f(bounds[3 + a]);
        const float ext = hi - lo;
        float f = ext > 0.0f ? (cc[a] - lo) / ext : 0.0f;
        f = fminf(fmaxf(f * 1024.0f, 0.0f), 1023.0f);
        q[a] = (uint32_t)f;
    }
    keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[i] = (uint32_t)i;
}

// ---- stable LSD radix sort, 8-bit digits -----------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_hist(const uint32_t* __restrict__ keys, int32_t n,
                                                       int shift, int32_t ntiles,
                                                       uint32_t* __restrict__ counts)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int32_t base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int32_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout, int32_t n,
                                                          int shift, int32_t ntiles,
                                                          const uint32_t* __restrict__ offsets)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcount[kSortThreads / kWave][256];
    run[threadIdx.x] = offsets[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int32_t base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        for (int w = 0; w < kSortThreads / kWave; ++w) wcount[w][threadIdx.x] = 0u;
        __syncthreads();
        const int32_t i = base + r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
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

// ---- binary radix tree ------------------------------------------------------------------
// Binary nodes live in the workspace; each stores both children's boxes, and in the spare
// lanes its own range of sorted triangles (a_hi.w = first, b_hi.w = count).
struct alignas(16) BinNode {
    float4 a_lo;  // xyz = child a box min, w = bits of child a (>= 0 node, < 0 leaf ~position)
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

__global__ __launch_bounds__(256) void k_tree(const uint32_t* __restrict__ k, int32_t n,
                                              BinNode* __restrict__ nodes,
                                              int32_t* __restrict__ parent)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(k, n, i, i - d);
    int32_t lmax = 2;
    while (delta(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int32_t l = 0;
    for (int32_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int32_t j = i + l * d;
    const int dnode = delta(k, n, i, j);
    int32_t s = 0;
    for (int32_t div = 2;; div <<= 1) {
        const int32_t t = (l + div - 1) / div;
        if (delta(k, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int32_t gamma = i + s * d + min(d, 0);
    const int32_t left = (min(i, j) == gamma) ? ~gamma : gamma;
    const int32_t right = (max(i, j) == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    const float inf = __int_as_float(0x7f800000);
    nodes[i].a_lo = make_float4(inf, inf, inf, __int_as_float(left));
    nodes[i].a_hi = make_float4(-inf, -inf, -inf, __int_as_float(min(i, j)));
    nodes[i].b_lo = make_float4(inf, inf, inf, __int_as_float(right));
    nodes[i].b_hi = make_float4(-inf, -inf, -inf, __int_as_float(max(i, j) - min(i, j) + 1));
    parent[left >= 0 ? left : (n - 1) + ~left] = i;
    parent[right >= 0 ? right : (n - 1) + ~right] = i;
}

__device__ inline float ld_coherent(const float* p)
{
    return __uint_as_float(__hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline void st_coherent(float* p, float v)
{
    __hip_atomic_store((uint32_t*)p, __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_leaves_refit(const float* __restrict__ v,
                                                      const int32_t* __restrict__ t, int32_t n,
                                                      const uint32_t* __restrict__ order,
                                                      float pad, BinNode* nodes,
                                                      BvhTri* __restrict__ out,
                                                      const int32_t* __restrict__ parent,
                                                      uint32_t* flags)
{
    const int32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const int32_t id = (int32_t)order[pos];
    const int64_t ia = t[3 * (int64_t)id], ib = t[3 * (int64_t)id + 1], ic = t[3 * (int64_t)id + 2];
    const float3 a = make_float3(v[3 * ia], v[3 * ia + 1], v[3 * ia + 2]);
    const float3 b = make_float3(v[3 * ib], v[3 * ib + 1], v[3 * ib + 2]);
    const float3 c = make_float3(v[3 * ic], v[3 * ic + 1], v[3 * ic + 2]);
    const float3 mn = make_float3(fminf(fminf(a.x, b.x), c.x), fminf(fminf(a.y, b.y), c.y),
                                  fminf(fminf(a.z, b.z), c.z));
    const float3 mx = make_float3(fmaxf(fmaxf(a.x, b.x), c.x), fmaxf(fmaxf(a.y, b.y), c.y),
                                  fmaxf(fmaxf(a.z, b.z), c.z));
    BvhTri tri;
    tri.v0 = make_float4(a.x, a.y, a.z, __int_as_float(id));
    tri.v1 = make_float4(b.x, b.y, b.z, 0.0f);
    tri.v2 = make_float4(c.x, c.y, c.z, 0.0f);
    out[pos] = tri;
    if (n == 1) return;
    const float pad2 = 2.0f * pad;
    float3 blo = make_float3(mn.x - pad2, mn.y - pad2, mn.z - pad2);
    float3 bhi = make_float3(mx.x + pad2, mx.y + pad2, mx.z + pad2);
    int32_t me = ~pos;
    int32_t p = parent[(n - 1) + pos];
    while (true) {
        BinNode* node = &nodes[p];
        const bool is_a = __float_as_int(node->a_lo.w) == me;
        float* slo = is_a ? &node->a_lo.x : &node->b_lo.x;
        float* shi = is_a ? &node->a_hi.x : &node->b_hi.x;
        st_coherent(slo, blo.x);
        st_coherent(slo + 1, blo.y);
        st_coherent(slo + 2, blo.z);
        st_coherent(shi, bhi.x);
        st_coherent(shi + 1, bhi.y);
        st_coherent(shi + 2, bhi.z);
        const uint32_t old = __hip_atomic_fetch_add(&flags[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0u) return;  // the sibling will finish this node
        const float* alo = &node->a_lo.x;
        const float* ahi = &node->a_hi.x;
        const float* bl = &node->b_lo.x;
        const float* bh = &node->b_hi.x;
        blo = make_float3(fminf(ld_coherent(alo), ld_coherent(bl)),
                          fminf(ld_coherent(alo + 1), ld_coherent(bl + 1)),
                          fminf(ld_coherent(alo + 2), ld_coherent(bl + 2)));
        bhi = make_float3(fmaxf(ld_coherent(ahi), ld_coherent(bh)),
                          fmaxf(ld_coherent(ahi + 1), ld_coherent(bh + 1)),
                          fmaxf(ld_coherent(ahi + 2), ld_coherent(bh + 2)));
        if (p == 0) return;
        me = p;
        p = parent[p];
    }
}

// ---- collapse into a 4-wide hierarchy ---------------------------------------------------
// For every binary node: start from its two children and repeatedly open the child with
// the largest surface area that holds more than kLeafMax triangles, until there are 4
// children or nothing left to open; children with at most kLeafMax triangles become leaf
// ranges (a radix-tree subtree always covers consecutive sorted triangles).  Each node's
// result depends only on its own subtree, so all nodes are collapsed in parallel; the ones
// reachable from the root form the hierarchy.
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

__global__ __launch_bounds__(256) void k_collapse4(const BinNode* __restrict__ nodes, int32_t n,
                                                   Bvh4Node* __restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
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
    const float inf = __int_as_float(0x7f800000);
    float lx[4], ly[4], lz[4], hx[4], hy[4], hz[4];
    int32_t cc[4];
    for (int q = 0; q < 4; ++q) {
        if (q < m) {
            lx[q] = s[q].lo.x; ly[q] = s[q].lo.y; lz[q] = s[q].lo.z;
            hx[q] = s[q].hi.x; hy[q] = s[q].hi.y; hz[q] = s[q].hi.z;
            cc[q] = s[q].count <= kLeafMax ? leaf_code(s[q].first, s[q].count) : s[q].code;
        } else {
            lx[q] = ly[q] = lz[q] = inf;
            hx[q] = hy[q] = hz[q] = -inf;
            cc[q] = kBvhEmptySlot;
        }
    }
    Bvh4Node o;
    o.lox = make_float4(lx[0], lx[1], lx[2], lx[3]);
    o.loy = make_float4(ly[0], ly[1], ly[2], ly[3]);
    o.loz = make_float4(lz[0], lz[1], lz[2], lz[3]);
    o.hix = make_float4(hx[0], hx[1], hx[2], hx[3]);
    o.hiy = make_float4(hy[0], hy[1], hy[2], hy[3]);
    o.hiz = make_float4(hz[0], hz[1], hz[2], hz[3]);
    o.child = make_int4(cc[0], cc[1], cc[2], cc[3]);
    o.unused = make_int4(0, 0, 0, 0);
    out[i] = o;
}

__global__ void k_header(BvhHeader* h, int32_t nt, float pad)
{
    h->nt = nt;
    h->root = nt <= kLeafMax ? (nt > 0 ? leaf_code(0, nt) : kBvhEmptySlot) : 0;
    h->pad = pad;
}

struct SortWork {
    uint32_t *k0, *v0, *k1, *v1, *counts, *bounds, *flags;
    int32_t* parent;
    BinNode* bin;
    void* scan;
    int32_t ntiles;
};

SortWork carve(void* work, int32_t nt)
{
    SortWork w;
    char* p = (char*)work;
    const size_t a = align256((size_t)nt * 4);
    w.ntiles = (int32_t)ceil_div(nt, kSortTile);
    w.k0 = (uint32_t*)p;
    p += a;
    w.v0 = (uint32_t*)p;
    p += a;
    w.k1 = (uint32_t*)p;
    p += a;
    w.v1 = (uint32_t*)p;
    p += a;
    w.counts = (uint32_t*)p;
    p += align256((size_t)w.ntiles * 256 * 4);
    w.bounds = (uint32_t*)p;
    p += 256;
    w.flags = (uint32_t*)p;
    p += align256((size_t)nt * 4);
    w.parent = (int32_t*)p;
    p += align256((size_t)(2 * (int64_t)nt) * 4);
    w.bin = (BinNode*)p;
    p += align256(sizeof(BinNode) * (size_t)nt);
    w.scan = p;
    return w;
}

}  // namespace

size_t bvh_bytes(int32_t nt)
{
    return 256 + sizeof(Bvh4Node) * bvh_node_count(nt) + sizeof(BvhTri) * (size_t)nt;
}

size_t bvh_work_bytes(int32_t nt)
{
    const int64_t ntiles = ceil_div(nt, kSortTile);
    return 4 * align256((size_t)nt * 4) + align256((size_t)ntiles * 256 * 4) + 256 +
           align256((size_t)nt * 4) + align256((size_t)(2 * (int64_t)nt) * 4) +
           align256(sizeof(BinNode) * (size_t)nt) + scan_work_bytes_u32(ntiles * 256);
}

hipError_t build_bvh(const float* verts, const int32_t* tris, int32_t nt, const rtsdf_grid& g,
                     void* bvh, void* work, hipStream_t s)
{
    const float pad = g.h * (1.0f / 256.0f);
    hipLaunchKernelGGL(k_header, dim3(1), dim3(1), 0, s, bvh_header(bvh), nt, pad);
    if (nt == 0) return hipGetLastError();
    SortWork w = carve(work, nt);
    const unsigned tb = (unsigned)ceil_div(nt, 256);
    hipLaunchKernelGGL(k_init, dim3(std::min<unsigned>(tb, 1024u)), dim3(256), 0, s, w.bounds,
                       w.flags, nt);
    hipLaunchKernelGGL(k_bounds, dim3(tb), dim3(256), 0, s, verts, tris, nt, w.bounds);
    hipLaunchKernelGGL(k_morton, dim3(tb), dim3(256), 0, s, verts, tris, nt, (const uint32_t*)w.bounds,
                       w.k0, w.v0);
    uint32_t *ka = w.k0, *va = w.v0, *kb = w.k1, *vb = w.v1;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_hist, dim3((unsigned)w.ntiles), dim3(kSortThreads), 0, s, ka, nt, shift,
                           w.ntiles, w.counts);
        hipError_t e = scan_exclusive_u32(w.counts, w.counts, (int64_t)w.ntiles * 256, nullptr, w.scan, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)w.ntiles), dim3(kSortThreads), 0, s, ka, va, kb, vb,
                           nt, shift, w.ntiles, (const uint32_t*)w.counts);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    BvhTri* out = bvh_tris(bvh, nt);
    if (nt > 1)
        hipLaunchKernelGGL(k_tree, dim3((unsigned)ceil_div(nt - 1, 256)), dim3(256), 0, s, ka, nt, w.bin,
                           w.parent);
    hipLaunchKernelGGL(k_leaves_refit, dim3(tb), dim3(256), 0, s, verts, tris, nt, va, pad, w.bin, out,
                       w.parent, w.flags);
    if (nt > 1)
        hipLaunchKernelGGL(k_collapse4, dim3((unsigned)ceil_div(nt - 1, 256)), dim3(256), 0, s,
                           (const BinNode*)w.bin, nt, bvh_nodes(bvh));
    return hipGetLastError();
}

}  // namespace rtsdf
