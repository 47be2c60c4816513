// Internal declarations shared by the HIP translation units of librtsdf.so.
// Host-side launchers return hipError_t; the C ABI layer (capi.cpp) validates arguments
// and turns errors into rtsdf_status codes.
#pragma once

#include "layout.h"

namespace rtsdf {

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

// One pass.  Between the first and the last pass of a call the buffers hold complemented ids
// (~id, EMPTY = 0: a load past the grid returns it for free); in_plain / out_plain say that
// the pass reads / writes the plain ids of the public format instead.
hipError_t jfa_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, bool in_plain, bool out_plain,
                    hipStream_t s);
// a pass whose input is mostly EMPTY (the offsets of at least a quarter of the longest side:
// the first two after voxelization) tests each plane's loaded ids for all-EMPTY first
bool jfa_sparse(const rtsdf_grid& g, int32_t k);
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
// the allocation-free variant's work cursors: a static device array per GPU
size_t raysample_scratch_bytes();
hipError_t raysample_scratch(void** out);
// frame_dev: when non-null, the frame index is read from it when the kernel runs (frame is
// then ignored)
hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list,
                     const int32_t* count, int64_t capacity, int32_t x, uint64_t key,
                     uint32_t frame, const uint32_t* frame_dev, uint32_t obj, float* dmin, uint32_t* hits,
                     uint64_t* argmin, void* work, hipStream_t s);

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


// ---- batched launchers ---------------------------------------------------------------

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
hipError_t shadow_forward_clip(const BatchView& hv, const float* fine, const rtsdf_shadow_ex& s, float* img,
                               hipStream_t st);
hipError_t shadow_backward_clip(const BatchView& hv, const float* fine, const rtsdf_shadow_ex& s,
                                const float* grad_img, float* grad_fine, hipStream_t st);
hipError_t clip_sample(const BatchView& hv, const float* fine, const float* pts, int64_t n, float* vals,
                       int32_t* levels, hipStream_t st);
hipError_t sdf_backward_batched(const BatchView& hv, const void* dplan, const float* grad_fine,
                                const uint32_t* hits, const uint64_t* argmin, const int32_t* list,
                                const int32_t* count, int64_t capacity, const void* bvh, const int32_t* tris,
                                int32_t x, uint64_t key, float* grad_verts, hipStream_t s);

}  // namespace rtsdf
