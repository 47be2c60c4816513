// One jump-flooding pass (section 2.2) over packed int32 seed ids.
//
// Query order: the stored seed first, then the 26 offsets e in {-1,0,1}^3 \ {0} in the
// order ez, ey, ex ascending.  A later query replaces the incumbent only when strictly
// closer, which is the same as taking the minimum of (d2, rank) for any rank that is
// increasing in that order: here rank 0 for the stored seed and 1 + L for the others,
// L = 9 (ez+1) + 3 (ey+1) + (ex+1) (so 1..13 and 15..27).
//
// Kernel: each thread owns one (x, y) column and walks the z positions of one residue
// class z = r + m*k (the only planes a pass with offset k couples), holding the 3 x 3
// neighbourhoods of planes m-1, m, m+1 in registers, so each output loads one new plane
// (9 values) instead of 27.  For every loaded seed s at column slot q = 3 (ey+1) + (ex+1)
// the thread precomputes
//     W = ((sx - px)^2 + (sy - py)^2 + sz^2) * 32 + 1 + q,
// and for output z = pz a candidate from plane ez has the signed 32-bit key
//     W + sz * (-64 pz) + 9 (ez+1) = (d2 - pz^2) * 32 + rank,
// an order-preserving image of (d2, rank): one v_mad_i32_i24 per candidate, each plane's
// nine keys reduced with v_min3_i32 before its rank offset 9 (ez+1) is added once (the
// stored seed takes its mid-plane key minus 1 + 4, i.e. rank 0).  The winner's id is reloaded from its (recently cached)
// position (the offset of each rank for the pass's k comes from a small LDS table, and the
// nine gathers of a plane are buffer loads off a scalar plane base).  EMPTY (-1) unpacks to (1023, 1023, 4095), which makes w - 2 pz sz >= 8.39e6
// > any real d2 (<= 3 * 1023^2), so it never wins against a seed; out-of-grid queries load
// EMPTY.  Keys stay within +-2^30.
#include "internal.h"
#include "tuning.h"

namespace rtsdf {

namespace {

constexpr int kBX = 64, kBY = RTSDF_JFA_ROWS;  // threads per block: 64 x-columns x kBY y-columns
constexpr int kChunk = RTSDF_JFA_CHUNK;        // lattice points per block along z
constexpr int kChunkSmall = 16;                // ... for passes that would launch few blocks
constexpr int64_t kFewBlocks = 2048;           // below this many blocks, use kChunkSmall
constexpr int32_t kEmptyV = 8000000;  // v >= this only for EMPTY

struct Cand {
    int32_t W;   // ((sx-px)^2 + (sy-py)^2 + sz^2) * 32 + 1 + q
    int32_t sz;
};

typedef short short2_t __attribute__((ext_vector_type(2)));

// (dx, dy) as packed int16 (|d| <= 1023) so that dx^2 + dy^2 + sz^2 is one v_dot2c_i32_i16
// on top of sz^2; all other factors are below 2^23, so the 24-bit multiplier is exact.
__device__ inline Cand prep(int32_t s, short2_t pxy, int32_t q)
{
    const uint32_t u = (uint32_t)s;
    const int32_t sz = (int32_t)(u >> 20);
    const short2_t sxy = __builtin_bit_cast(short2_t, (u & 1023u) | (((u >> 10) & 1023u) << 16));
    const short2_t d = sxy - pxy;
    return Cand{__builtin_amdgcn_sdot2(d, d, __mul24(sz, sz), false) * 32 + (1 + q), sz};
}

__device__ inline int32_t cand_key(Cand c, int32_t m64pz) { return c.W + __mul24(c.sz, m64pz); }

__device__ inline int32_t min9(const int32_t* k)
{
    return min(min(min(k[0], k[1]), k[2]), min(min(min(k[3], k[4]), k[5]), min(min(k[6], k[7]), k[8])));
}

// element offset, relative to the output point, of the query that rank rk names, for
// offset k (the winner's id is reloaded from there); built once per work-group in LDS:
// rank 0 is the point itself, rank 1 + L the query L = 9 (ez+1) + 3 (ey+1) + (ex+1)
__device__ inline void rank_table(int32_t* tab, int32_t nx, int32_t ny, int32_t k)
{
    const int t = threadIdx.x + threadIdx.y * kBX;
    if (t < 28) {
        const int32_t L = t == 0 ? 13 : t - 1;
        const int32_t ez = L / 9 - 1, ey = (L / 3) % 3 - 1, ex = L % 3 - 1;
        tab[t] = ex * k + ey * k * nx + ez * k * (nx * ny);
    }
}

// One plane of the input as a buffer resource: a scalar base and 32-bit byte offsets, so
// the nine gathers of a plane need no per-lane address arithmetic.
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const int32_t* in, uint32_t plane, int32_t z)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)(in + (size_t)plane * (uint32_t)z), (short)0, 0x7FFFFFFF,
                                            0x00020000);
}

// work-group (bx, by, bz) of a pass over one grid: x-columns bx*64.., y-columns by*4..,
// residue class r and chunk c of that class from bz; tab = rank_table(nx, ny, k)
template <int kCh>
__device__ __forceinline__ void jfa_block(const int32_t* __restrict__ in, int32_t* __restrict__ out, int32_t nx,
                                          int32_t ny, int32_t nz, int32_t k, int32_t chunks_per_residue,
                                          int32_t bx, int32_t by, int32_t bz, const int32_t* tab)
{
    const int32_t x = bx * kBX + threadIdx.x;
    const int32_t y = by * kBY + threadIdx.y;
    const int32_t r = bz / chunks_per_residue;
    const int32_t c = bz - r * chunks_per_residue;
    if (x >= nx || y >= ny || r >= nz) return;
    const int32_t mcount = (nz - r + k - 1) / k;  // lattice points z = r + m k < nz
    const int32_t m0 = c * kCh;
    if (m0 >= mcount) return;
    const int32_t m1 = min(m0 + kCh, mcount);
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;  // grids hold at most 2^30 points

    // byte offsets of the 3 x 3 neighbourhood columns; out-of-grid columns read EMPTY
    uint32_t off[9];
    bool ok[9];
#pragma unroll
    for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
        for (int ex = -1; ex <= 1; ++ex) {
            const int q = 3 * (ey + 1) + (ex + 1);
            const int32_t qx = x + ex * k, qy = y + ey * k;
            ok[q] = qx >= 0 && qx < nx && qy >= 0 && qy < ny;
            off[q] = ok[q] ? 4u * ((uint32_t)qx + (uint32_t)nx * (uint32_t)qy) : 0u;  // bytes
        }

    const short2_t pxy = __builtin_bit_cast(short2_t, (uint32_t)x | ((uint32_t)y << 16));
    // planes outside the grid (m < 0 or z >= nz, uniform) load a valid plane and read EMPTY
    auto load_plane = [&](int32_t m, Cand* dst) {
        const int32_t z = r + m * k;
        const bool pv = m >= 0 && z < nz;
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in, plane, pv ? z : r);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off[q], 0, 0);
            dst[q] = prep(ok[q] && pv ? v : RTSDF_EMPTY, pxy, q);
        }
    };
    const uint32_t pxy_idx = (uint32_t)x + (uint32_t)nx * (uint32_t)y;
    // output for lattice point m from planes m-1 (lo), m (mid), m+1 (hi)
    auto emit = [&](int32_t m, const Cand* lo, const Cand* mid, const Cand* hi) {
        const int32_t pz = r + m * k;
        const int32_t m64pz = -64 * pz;
        int32_t a[9], b[9], c[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            a[q] = cand_key(lo[q], m64pz);
            b[q] = cand_key(mid[q], m64pz);
            c[q] = cand_key(hi[q], m64pz);
        }
        const int32_t self = b[4] - 5;  // the stored seed: rank 0 instead of 1 + 4
        const int32_t mid8 = min(min(min(b[0], b[1]), b[2]), min(min(b[3], b[5]), min(min(b[6], b[7]), b[8])));
        const int32_t best = min(min(min9(a), mid8 + 9), min(min9(c) + 18, self));
        const uint32_t p = pxy_idx + plane * (uint32_t)pz;
        int32_t id = RTSDF_EMPTY;
        if ((best >> 5) < kEmptyV) id = in[(uint32_t)((int32_t)p + tab[best & 31])];
        out[p] = id;
    };

    Cand A[9], B[9], C[9];
    load_plane(m0 - 1, A);
    load_plane(m0, B);
    // rotate the three plane buffers by unrolling three outputs per trip
    for (int32_t m = m0; m < m1; m += 3) {
        load_plane(m + 1, C);
        emit(m, A, B, C);
        if (m + 1 >= m1) break;
        load_plane(m + 2, A);
        emit(m + 1, B, C, A);
        if (m + 2 >= m1) break;
        load_plane(m + 3, B);
        emit(m + 2, C, A, B);
    }
}

template <int kCh>
__global__ __launch_bounds__(kBX * kBY) void k_jfa_stream(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int32_t nx,
                                                          int32_t ny, int32_t nz, int32_t k,
                                                          int32_t chunks_per_residue)
{
    __shared__ int32_t tab[32];
    rank_table(tab, nx, ny, k);
    __syncthreads();
    jfa_block<kCh>(in, out, nx, ny, nz, k, chunks_per_residue, blockIdx.x, blockIdx.y, blockIdx.z, tab);
}

__host__ __device__ inline int32_t chunks_per_residue(int32_t nz, int32_t k, int32_t chunk = kChunk)
{
    return (int32_t)ceil_div(ceil_div(nz, k), chunk);
}

// One pass over every object still flooding: the flat work-group index picks the object
// from this pass's prefix table, then the object's own geometry and offset; object o reads
// the buffer holding its pass-p input (its start buffer alternates with p).
__global__ __launch_bounds__(kBX * kBY) void k_jfa_batched(const char* __restrict__ plan, int32_t nobj,
                                                           int32_t pass, int32_t* __restrict__ seeds,
                                                           int32_t* __restrict__ scratch)
{
    const BatchView v = batch_view(plan, nobj);
    const int32_t* prefix = v.pass_prefix + (int64_t)pass * (nobj + 1);
    const int32_t b = blockIdx.x;
    const int32_t o = find_object(prefix, nobj, b);
    const BatchObject& ob = v.obj[o];
    const int32_t k = jfa_offset(ob.k0, ob.nhalf, pass);
    const int32_t nx = ob.g.nx, ny = ob.g.ny, nz = ob.g.nz;
    const int32_t gx = (nx + kBX - 1) / kBX, gy = (ny + kBY - 1) / kBY;
    const int32_t l = b - prefix[o];
    const bool from_scratch = (ob.flip ^ (pass & 1)) != 0;
    const int32_t* in = (from_scratch ? scratch : seeds) + ob.vox_off;
    int32_t* out = (from_scratch ? seeds : scratch) + ob.vox_off;
    __shared__ int32_t tab[32];
    rank_table(tab, nx, ny, k);
    __syncthreads();
    jfa_block<kChunk>(in, out, nx, ny, nz, k, chunks_per_residue(nz, k), l % gx, (l / gx) % gy, l / (gx * gy), tab);
}

}  // namespace

int64_t jfa_pass_blocks(const rtsdf_grid& g, int32_t k)
{
    return ceil_div(g.nx, kBX) * ceil_div(g.ny, kBY) * std::min<int64_t>(k, g.nz) * chunks_per_residue(g.nz, k);
}

hipError_t jfa_batched_pass(const BatchView& hv, const void* dplan, int32_t* seeds, int32_t* scratch, int32_t pass,
                            hipStream_t s)
{
    const int32_t blocks = hv.h->pass_blocks[pass];
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jfa_batched, dim3((unsigned)blocks), dim3(kBX, kBY), 0, s, (const char*)dplan,
                       hv.h->nobj, pass, seeds, scratch);
    return hipGetLastError();
}

hipError_t jfa_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, hipStream_t s)
{
    const int64_t residues = std::min<int64_t>(k, g.nz);
    const bool few = jfa_pass_blocks(g, k) < kFewBlocks;  // small grids: shorter chunks, more blocks
    const int64_t per_res = chunks_per_residue(g.nz, k, few ? kChunkSmall : kChunk);
    dim3 grid((unsigned)ceil_div(g.nx, kBX), (unsigned)ceil_div(g.ny, kBY), (unsigned)(residues * per_res));
    if (few)
        hipLaunchKernelGGL(k_jfa_stream<kChunkSmall>, grid, dim3(kBX, kBY), 0, s, in, out, g.nx, g.ny, g.nz, k,
                           (int32_t)per_res);
    else
        hipLaunchKernelGGL(k_jfa_stream<kChunk>, grid, dim3(kBX, kBY), 0, s, in, out, g.nx, g.ny, g.nz, k,
                           (int32_t)per_res);
    return hipGetLastError();
}

}  // namespace rtsdf
