// Internal declarations shared by the HIP translation units of librtsdf.so.
// Host-side launchers return hipError_t; the C ABI layer (capi.cpp) validates arguments
// and turns errors into rtsdf_status codes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rtsdf.h"

namespace rtsdf {

constexpr int kWave = 64;

__host__ __device__ inline int64_t nvox(const rtsdf_grid& g) { return (int64_t)g.nx * g.ny * g.nz; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Number of work-groups that keeps every CU of the device busy for grid-stride kernels.
int persistent_groups(int threads_per_group);

// ---- exclusive prefix sums (scan.hip) -------------------------------------------------
// out[i] = sum(in[0..i)); *total = sum(in[0..n)) if total != nullptr.  out may alias in.
size_t scan_work_bytes_u32(int64_t n);
size_t scan_work_bytes_u64(int64_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                              void* work, hipStream_t s);
hipError_t scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                              void* work, hipStream_t s);

// ---- module launchers -----------------------------------------------------------------
size_t voxelize_work_bytes(int32_t nt);
hipError_t voxelize(const float* verts, const int32_t* tris, int32_t nt, const rtsdf_grid& g,
                    int32_t* seeds, void* work, hipStream_t s);

hipError_t jfa_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k,
                    hipStream_t s);
int64_t jfa_pass_blocks(const rtsdf_grid& g, int32_t k);  // work-groups of one pass

size_t band_work_bytes(const rtsdf_grid& g);
hipError_t band(const int32_t* seeds, const rtsdf_grid& g, int32_t band_vox, int32_t* list,
                int32_t* count, void* work, hipStream_t s);
// mask of the grid refined by r over `coarse` (section 2.3 on a finer traced grid)
size_t band_refined_work_bytes(const rtsdf_grid& coarse, int32_t r);
hipError_t band_refined(const int32_t* seeds, const rtsdf_grid& coarse, int32_t r, int32_t band_vox,
                        int32_t* list, int32_t* count, void* work, hipStream_t s);

size_t bvh_bytes(int32_t nt);
constexpr int kBvhSortTile = 1024;  // triangles per sort tile of the hierarchy build
size_t bvh_work_bytes(int64_t total_tris, int64_t total_tiles, int32_t nobj);
inline size_t bvh_work_bytes(int32_t nt) { return bvh_work_bytes(nt, ceil_div(nt, kBvhSortTile), 1); }
hipError_t build_bvh(const float* verts, const int32_t* tris, int32_t nt, const rtsdf_grid& g,
                     void* bvh, void* work, int32_t method, hipStream_t s);

hipError_t reset_accum(float* dmin, uint32_t* hits, uint64_t* argmin, int64_t n, hipStream_t s);
size_t raysample_work_bytes(int64_t capacity, int32_t x);
hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list,
                     const int32_t* count, int64_t capacity, int32_t x, uint64_t key,
                     uint32_t frame, uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin,
                     void* work, hipStream_t s);

hipError_t combine(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& g,
                   int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                   int32_t first_frame, int32_t consume, float* state, float* fine,
                   hipStream_t s);
hipError_t combine_refined(const int32_t* seeds, float* dmin, uint32_t* hits, const rtsdf_grid& coarse, int32_t r,
                           int32_t band_vox, float beta, float bias, int32_t mode, float alpha,
                           int32_t first_frame, int32_t consume, float* state, float* fine, hipStream_t s);

hipError_t shadow_forward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s, float* img,
                          hipStream_t st);
hipError_t shadow_backward(const float* fine, const rtsdf_grid& g, const rtsdf_shadow& s,
                           const float* grad_img, float* grad_fine, hipStream_t st);
hipError_t shadow_forward_ex(const float* fine, const rtsdf_grid& g, const rtsdf_shadow_ex& s, float* img,
                             hipStream_t st);
hipError_t shadow_backward_ex(const float* fine, const rtsdf_grid& g, const rtsdf_shadow_ex& s,
                              const float* grad_img, float* grad_fine, hipStream_t st);
hipError_t sdf_backward(const float* grad_fine, const uint32_t* hits, const uint64_t* argmin,
                        const int32_t* list, const int32_t* count, int64_t capacity, const void* bvh,
                        const int32_t* tris, const rtsdf_grid& g, int32_t x, uint64_t key, uint32_t obj,
                        float* grad_verts, hipStream_t s);

// ---- batched objects (batch.cpp builds the plan; kernels read its device copy) ----------
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

size_t band_batched_work_bytes(int64_t total_vox);
hipError_t voxelize_batched(const BatchView& hv, const void* dplan, const float* verts, const int32_t* tris,
                            int32_t* seeds, int32_t* scratch, void* work, hipStream_t s);
hipError_t jfa_batched_pass(const BatchView& hv, const void* dplan, int32_t* seeds, int32_t* scratch, int32_t pass,
                            hipStream_t s);
hipError_t band_batched(const BatchView& hv, const void* dplan, const int32_t* seeds, int32_t* list,
                        int32_t* count, void* work, hipStream_t s);
hipError_t combine_batched(const BatchView& hv, const void* dplan, const int32_t* seeds, const float* dmin,
                           const uint32_t* hits, float* fine, hipStream_t s);
hipError_t raysample_batched(const BatchView& hv, const void* dplan, const void* bvh, const int32_t* list,
                             const int32_t* count, int64_t capacity, int32_t x, uint64_t key, uint32_t frame,
                             float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s);
hipError_t build_bvh_batched(const BatchView& hv, const void* dplan, const float* verts, const int32_t* tris,
                             void* bvh, void* work, int32_t method, hipStream_t s);
hipError_t sdf_backward_batched(const BatchView& hv, const void* dplan, const float* grad_fine,
                                const uint32_t* hits, const uint64_t* argmin, const int32_t* list,
                                const int32_t* count, int64_t capacity, const void* bvh, const int32_t* tris,
                                int32_t x, uint64_t key, float* grad_verts, hipStream_t s);

// ---- BVH blob layout (lbvh.hip writes it, raysample.hip reads it) ----------------------
// [header 256 B][4-wide nodes: max(nt-1, 1) x Bvh4Node][triangles: nt x BvhTri]
// A 4-wide node is stored at the index of the binary radix-tree node it was collapsed
// from (only some indices are reachable).  Child codes: c >= 0 is a node index,
// kBvhEmptySlot an unused slot, any other c < 0 a leaf range ~c = first | (count-1) << 26
// of `count` (1..kLeafMax) consecutive triangles in sorted order.
constexpr int32_t kBvhEmptySlot = (int32_t)0x80000000;
constexpr int kLeafMax = 3;

struct BvhHeader {
    int32_t nt;
    int32_t root;     // child code of the root (a node, or a leaf range when nt <= kLeafMax)
    float pad;        // hit-test widening (h / 256)
    int32_t reserved[61];
};
struct alignas(16) Bvh4Node {  // structure of arrays over the 4 children
    float4 lox, loy, loz;
    float4 hix, hiy, hiz;
    int4 child;
    int4 unused;
};
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
