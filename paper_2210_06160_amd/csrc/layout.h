// Data layouts shared by the kernels and the host code of librtsdf.so: the batch plan
// (capi.cpp builds it, the batched kernels read its device copy) and the hierarchy blob
// (lbvh.hip writes it, raysample.hip and backward.hip read it).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rtsdf.h"
#include "tuning.h"

namespace rtsdf {

constexpr int kWave = 64;

__host__ __device__ inline int64_t nvox(const rtsdf_grid& g) { return (int64_t)g.nx * g.ny * g.nz; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---- batched objects (capi.cpp builds the plan; kernels read its device copy) ----------
// Plan bytes (identical on host and device): BatchHeader, then nobj BatchObject entries,
// then vox_prefix int64[nobj + 1], tri_prefix int32[nobj + 1] and, for every JFA pass p,
// pass_prefix int32[nobj + 1] (work-groups of the objects still flooding at pass p).
constexpr int64_t kBatchAlign = RTSDF_BATCH_ALIGN;  // voxels; one mask / combine tile
constexpr int kMaxPasses = 19;                      // 10 halving passes + 8 extra + 1

struct BatchObject {
    rtsdf_grid g;
    int32_t band_vox;
    int64_t vox_off;   // first grid point in the concatenated grids (multiple of kBatchAlign)
    int64_t bvh_off;   // byte offset of the object's hierarchy (multiple of 256)
    int32_t vert_off, tri_off;
    int32_t nv, nt;
    int32_t nsteps;    // JFA passes: the halving offsets k0 .. 1, then `extra` passes of 1
    int32_t nhalf;     // number of halving passes
    int32_t k0;
    int32_t flip;      // initial seeds go to the second buffer (nsteps odd)
    float beta, bias;
    int32_t tile_off;  // first hierarchy-build sort tile (tiles of kBvhSortTile triangles)
    int32_t reserved;
};

struct BatchHeader {
    uint32_t magic;
    int32_t nobj;
    int32_t max_passes;
    int32_t reserved0;
    int64_t total_vox, total_verts, total_tris;  // total_tris < 2^26
    uint64_t bvh_bytes;
    uint64_t plan_bytes;
    const void* device;   // the device copy of these bytes
    int32_t pass_blocks[kMaxPasses];  // JFA work-groups per pass (host launch sizes)
    int32_t total_tiles;              // hierarchy-build sort tiles of all objects
    int32_t reserved[256 / 4 - 17 - kMaxPasses];
};
static_assert(sizeof(BatchHeader) == 256, "batch header is 256 bytes");
constexpr uint32_t kBatchMagic = 0x52534442u;  // "BDSR"

inline size_t batch_plan_bytes(int32_t nobj)
{
    return sizeof(BatchHeader) + sizeof(BatchObject) * (size_t)nobj + 8 * (size_t)(nobj + 1) +
           4 * (size_t)(nobj + 1) * (1 + kMaxPasses);
}
struct BatchView {  // typed pointers into a plan (host or device copy)
    const BatchHeader* h;
    const BatchObject* obj;
    const int64_t* vox_prefix;
    const int32_t* tri_prefix;
    const int32_t* pass_prefix;  // [max_passes][nobj + 1]
};
__host__ __device__ inline BatchView batch_view(const void* plan, int32_t nobj)
{
    BatchView v;
    const char* p = (const char*)plan;
    v.h = (const BatchHeader*)p;
    p += sizeof(BatchHeader);
    v.obj = (const BatchObject*)p;
    p += sizeof(BatchObject) * (size_t)nobj;
    v.vox_prefix = (const int64_t*)p;
    p += 8 * (size_t)(nobj + 1);
    v.tri_prefix = (const int32_t*)p;
    p += 4 * (size_t)(nobj + 1);
    v.pass_prefix = (const int32_t*)p;
    return v;
}
// last o in [0, nobj) with prefix[o] <= i (prefix ascending, prefix[0] = 0)
template <typename T>
__host__ __device__ inline int32_t find_object(const T* prefix, int32_t nobj, T i)
{
    int32_t lo = 0, hi = nobj - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// JFA offset of pass p for an object whose halving offsets are k0, k0/2, .., 1 (nhalf of
// them) followed by passes of offset 1
__host__ __device__ inline int32_t jfa_offset(int32_t k0, int32_t nhalf, int32_t p)
{
    return p < nhalf ? (k0 >> p) : 1;
}

// ---- BVH blob layout (lbvh.hip writes it, raysample.hip and backward.hip read it) --------
// [header 256 B][4-wide nodes: max(nt-1, 1) x Bvh4Node][triangles: nt x BvhTri]
// A 4-wide node is stored at the index of the binary radix-tree node it was collapsed
// from (only some indices are reachable).  Child codes: c >= 0 is a node index,
// kBvhEmptySlot an unused slot, any other c < 0 a leaf range ~c = first | (count-1) << 26
// of `count` (1..kLeafMax) consecutive triangles in sorted order.
constexpr int32_t kBvhEmptySlot = (int32_t)0x80000000;
// Triangles of one hierarchy: at most 2^26 (the leaf code's first field); fewer than 2^26
// nodes keep a node's byte offset (node * 64) within 32 bits, which traversal relies on.
constexpr int32_t kBvhMaxTris = 1 << 26;
constexpr int kLeafMax = RTSDF_LEAF_MAX;

struct BvhHeader {
    int32_t nt;
    int32_t root;     // child code of the root (a node, or a leaf range when nt <= kLeafMax)
    float pad;        // hit-test widening (h / 256)
    int32_t depth;    // 4-wide nodes on the longest root-to-leaf path (0: the root is a leaf)
    int32_t reserved[60];
};
// A traversal pushes at most 3 entered siblings per node on its path plus one leaf range,
// so its stack holds at most 3 * depth + 1 entries; rays through a deeper hierarchy (a
// clustering tree has no depth bound; the radix tree's is 56) test every triangle instead,
// which returns the same closest hit.
constexpr int kMaxStack = 176;
__host__ __device__ inline bool bvh_too_deep(int32_t depth) { return 3 * depth + 1 > kMaxStack; }
// A 4-wide node (64 bytes).  The children's boxes are quantised to 8 bits per plane on a
// grid anchored at the node box's low corner o with a power-of-two step s per axis: child
// q's low plane on axis a is o_a + s_a * byte q of lo[a], its high plane o_a + s_a * byte q
// of hi[a].  Low planes are rounded down and high planes up (in exact arithmetic), so each
// quantised box contains its child's box.  Unused slots (code kBvhEmptySlot) hold lo bytes
// 255 and hi bytes 0; traversal rejects them by their code.
struct alignas(64) Bvh4Node {
    float ox, oy, oz;   // o: the node box's low corner
    uint32_t exps;      // biased exponents of the steps: s_a = 2^(e_a - 127), e = ex | ey << 8 | ez << 16
    int4 child;
    uint32_t lo[3];     // byte q: child q's low plane on x, y, z
    uint32_t hi[3];     // byte q: child q's high plane on x, y, z
    uint32_t unused[2];
};
static_assert(sizeof(Bvh4Node) == 64, "node size");
struct alignas(16) BvhTri {   // triangle in sorted (leaf) order
    float4 v0;    // xyz = v0, w = bits of the original triangle index
    float4 v1;    // xyz = v1
    float4 v2;    // xyz = v2
};

__host__ __device__ inline int32_t leaf_code(int32_t first, int32_t count)
{
    return ~(first | ((count - 1) << 26));
}
__host__ __device__ inline int32_t leaf_first(int32_t code) { return (~code) & 0x3FFFFFF; }
__host__ __device__ inline int32_t leaf_count(int32_t code) { return ((~code) >> 26) + 1; }

inline size_t bvh_node_count(int32_t nt) { return (size_t)(nt > 1 ? nt - 1 : 1); }
inline BvhHeader* bvh_header(void* b) { return (BvhHeader*)b; }
inline Bvh4Node* bvh_nodes(void* b) { return (Bvh4Node*)((char*)b + 256); }
inline BvhTri* bvh_tris(void* b, int32_t nt) {
    return (BvhTri*)((char*)b + 256 + sizeof(Bvh4Node) * bvh_node_count(nt));
}

}  // namespace rtsdf
