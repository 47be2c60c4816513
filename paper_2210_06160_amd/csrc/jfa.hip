// One jump-flooding pass (section 2.2) over packed int32 seed ids.
//
// Query order: the stored seed first, then the 26 offsets e in {-1,0,1}^3 \ {0} in the
// order ez, ey, ex ascending.  A later query replaces the incumbent only when strictly
// closer, which is the same as taking the minimum of (d2, rank) for any rank that is
// increasing in that order: here rank 0 for the stored seed and 1 + L for the others,
// L = 9 (ez+1) + 3 (ey+1) + (ex+1) (so 1..13 and 15..27).
//
// Internal ids.  Between the first and the last pass of a call the buffers hold the
// complement c = ~id of each packed id (EMPTY = -1 becomes 0); its fields are the
// complemented coordinates (cx, cy, cz) = (1023 - x, 1023 - y, 4095 - z), and distances
// between complemented points equal the true ones.  A load past a plane returns 0, i.e.
// EMPTY, so neighbours outside the grid cost nothing (see Column).  The first pass
// complements what it loads, the last stores plain ids again.
//
// Keys.  For a seed c loaded at column slot q = 3 (ey+1) + (ex+1) of a thread's column,
// complemented (qx, qy), the thread computes once
//     W = ((cx - qx)^2 + (cy - qy)^2 + cz^2) * 32 + 1 + q,
// and for an output at z = pz (complemented pz' = 4095 - pz) the candidate's signed 32-bit
// key is
//     W + cz * (-64 pz') + 9 (ez+1) = (d2 - pz'^2) * 32 + rank,
// an order-preserving image of (d2, rank): one v_mad_i32_i24 per candidate.  A plane's
// keys for one output are reduced (v_min3_i32) before that plane's rank offset 9 (ez+1)
// is added once; the stored seed takes its mid-plane key minus 1 + 4 (rank 0).  The
// winner's id is reloaded from the query its rank names (offsets from a 28-entry LDS
// table per work-group).  Grids have at most 1024 points a side, so a real seed has
// d2 <= 3 * 1023^2 < 3072^2 <= pz'^2 and a negative key, while EMPTY (c = 0, the point
// (1023, 1023, 4095)) has d2 >= pz'^2 and a key >= 0: it never wins against a seed, and a
// minimum >= 0 means no seed was seen.  Keys lie in (-2^30, 2^29.3).
//
// Streaming.  A pass with offset k couples only the z positions of one residue class
// z = r + m k.  Each thread owns one (x, y) column and walks the lattice points m of a
// residue class in order; plane m contributes to outputs m + 1 (as their ez = -1 plane),
// m (ez = 0, and the stored seed) and m - 1 (ez = +1), so each plane is loaded and its W
// computed once for up to three outputs, held only as three running minima.  Which of the
// three roles a plane has is fixed per work-group (first and last planes of a chain have
// one or two), so each role set is its own instantiation.
//
// Out-of-grid neighbours: a neighbour column (x + ex k, y + ey k) outside the grid loads the
// thread's own column and is OR-ed with an all-ones mask, which makes it EMPTY (no select,
// no branch); a plane outside the grid is never loaded (the chain's first and last planes
// have fewer roles).  When k >= ny (or k >= nx) the ey = +-1 rows (ex = +-1 columns) are
// outside for every point and are dropped at compile time.  In the sparse early passes
// (mostly EMPTY input, RTSDF_JFA_SPARSE) a plane's arithmetic is skipped when every id it
// loaded is EMPTY on every lane of the wave.  None of this changes any result.
//
// Work distribution.  A work-group is 64 RTSDF_JFA_WAVES consecutive columns of a plane
// (x fastest, across row ends, so no lane idles at the end of a row; rows taken in the
// order of their residue mod k when rows k apart would otherwise be far apart in launch
// order, see pass_row) and a z task: a chunk of one residue class's lattice points, or,
// when classes are short (large k), several whole classes, so that per-group set-up is
// spread over about RTSDF_JFA_CHUNK outputs per thread.  Work-groups are dealt to the 8
// XCDs round-robin in launch order; the launch index is remapped so that each XCD runs one
// contiguous range of tasks (z-major), so the planes and rows that a task's neighbours read
// are fetched into one XCD's L2 rather than into several.
#include "internal.h"
#include "tuning.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 64 * RTSDF_JFA_WAVES;  // threads (= consecutive columns of a plane) per work-group
constexpr int kChunk = RTSDF_JFA_CHUNK;        // outputs per thread and work-group along z
constexpr int kChunkSmall = 16;                // ... for passes that would launch few blocks
constexpr int64_t kFewBlocks = 2048;           // below this many blocks, use kChunkSmall
constexpr int kXcds = 8;
constexpr int32_t kNoKey = 0x7F000000;  // no candidate yet: above every key, and + 18 does not overflow
constexpr uint32_t kOutside = 0x80000000u;  // buffer offset past every plane: the load returns 0

struct Cand {
    int32_t W;   // ((cx-qx)^2 + (cy-qy)^2 + cz^2) * 32 + 1 + q, in complemented coordinates
    int32_t cz;
};

typedef short short2_t __attribute__((ext_vector_type(2)));

// c = ~id of a loaded seed (0 for EMPTY): its fields are the complemented coordinates
// (1023 - sx, 1023 - sy, 4095 - sz).  (dx, dy) as packed int16 (|d| <= 1023) so that
// dx^2 + dy^2 + cz^2 is one v_dot2c_i32_i16 on top of cz^2; all other factors are below
// 2^23, so the 24-bit multiplier is exact.
__device__ inline Cand prep(uint32_t c, short2_t qxy, int32_t q)
{
    const int32_t cz = (int32_t)(c >> 20);
    uint32_t cy = c & 0xFFC00u;
    asm("" : "+v"(cy));  // keeps the double-rate AND before the shift (one v_lshl_or below)
    const short2_t cxy = __builtin_bit_cast(short2_t, (cy << 6) | (c & 1023u));
    const short2_t d = cxy - qxy;
    return Cand{__builtin_amdgcn_sdot2(d, d, __mul24(cz, cz), false) * 32 + (1 + q), cz};
}

// m = -64 (4095 - pz): the key W + cz m = (d^2 - (4095 - pz)^2) 32 + rank
__device__ inline int32_t cand_key(Cand c, int32_t m) { return c.W + __mul24(c.cz, m); }
__device__ inline int32_t key_factor(int32_t z) { return 64 * z - 64 * 4095; }

__device__ inline int32_t min9(const int32_t* k)
{
    return min(min(min(k[0], k[1]), k[2]), min(min(min(k[3], k[4]), k[5]), min(min(k[6], k[7]), k[8])));
}

// element offset, relative to the output point, of the query that rank rk names, for
// offset k (the winner's id is reloaded from there); built once per work-group in LDS:
// rank 0 is the point itself, rank 1 + L the query L = 9 (ez+1) + 3 (ey+1) + (ex+1)
__device__ inline void rank_table(int32_t* tab, int32_t nx, int32_t ny, int32_t k)
{
    const int t = threadIdx.x;
    if (t < 28) {
        const int32_t L = t == 0 ? 13 : t - 1;
        const int32_t ez = L / 9 - 1, ey = (L / 3) % 3 - 1, ex = L % 3 - 1;
        tab[t] = ex * k + ey * k * nx + ez * k * (nx * ny);
    }
}

// One plane of the input as a buffer resource: a scalar base and 32-bit byte offsets, so
// the gathers of a plane need no per-lane address arithmetic; its size is the plane's, so a
// load at an offset past it (kOutside) returns 0 without touching memory.
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const int32_t* in, uint32_t plane, int32_t z)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)(in + (size_t)plane * (uint32_t)z), (short)0,
                                            (int)(4u * plane), 0x00020000);
}

// Rows of a plane in the order a pass walks them: grouped by their residue mod k (rows rho,
// rho + k, rho + 2k, ... one after the other), so that the work-groups reading a row as their
// own and as their y -/+ k neighbour row run at about the same time on one XCD and share
// its L2; in plain order they are k nx / kThreads work-groups apart.  Identity when k = 1 or
// k >= ny, and kept plain when rows k apart lie within kNearBlocks work-groups anyway.
constexpr int64_t kNearBlocks = 32;

__device__ inline int32_t pass_row(int32_t i, int32_t nx, int32_t ny, int32_t k)
{
    if ((int64_t)k * nx <= kNearBlocks * kThreads || k >= ny) return i;
    const int32_t c0 = ny / k, r = ny - c0 * k;  // residues rho < r have c0 + 1 rows, the others c0
    const int32_t split = r * (c0 + 1);
    int32_t rho, j;
    if (i < split) {
        rho = i / (c0 + 1);
        j = i - rho * (c0 + 1);
    } else {
        const int32_t i2 = i - split;
        rho = r + i2 / c0;
        j = i2 - (rho - r) * c0;
    }
    return rho + j * k;
}

// z tasks of one pass: either chunks of at most kCh lattice points of one residue class
// (per_res > 1 chunks of equal length `len` per class, one class per task), or about `group`
// whole classes per task, task t taking classes t, t + count, t + 2 count, ...  Both keep
// the work of the XCDs' contiguous task ranges equal: the classes r < nz mod k hold one
// lattice point more than the others, and taking them in consecutive groups would hand
// them all to the first XCDs.
struct ZTasks {
    int32_t res;      // residue classes: min(k, nz)
    int32_t per_res;  // chunks per class (>= 1)
    int32_t len;      // lattice points per chunk (when per_res > 1)
    int32_t group;    // classes per task, at most (>= 1; > 1 only when per_res == 1)
    int32_t count;    // tasks
};

__host__ __device__ inline ZTasks z_tasks(int32_t nz, int32_t k, int32_t ch)
{
    ZTasks t;
    t.res = k < nz ? k : nz;
    const int32_t mmax = (nz + k - 1) / k;  // lattice points of class 0 (the longest)
    t.per_res = (mmax + ch - 1) / ch;
    t.len = (mmax + t.per_res - 1) / t.per_res;
    t.group = t.per_res > 1 ? 1 : (ch / mmax > 1 ? ch / mmax : 1);
    t.count = t.per_res > 1 ? t.res * t.per_res : (t.res + t.group - 1) / t.group;
    return t;
}

// What a thread knows about its column for one pass: for each of the 3 x 3 neighbour
// columns q, its byte offset within a plane, kOutside when the column lies outside the grid
// (the load returns 0: EMPTY in complemented ids), and its complemented (x, y).  A pass
// whose input holds plain ids loads its own column instead and ORs the mask inv (all ones
// outside) into the id before complementing it, which gives 0 there too.
template <bool kInC>
struct Column {
    uint32_t off[9];
    int32_t inv[9];
    short2_t qxy;
};

// Neighbour rows / columns a pass can reach anywhere in the grid: 3, or only the middle one
// when the offset is at least the grid's extent on that axis.
template <int kRows, int kCols>
struct Slots {
    static constexpr bool has(int q) { return (kRows == 3 || q / 3 == 1) && (kCols == 3 || q % 3 == 1); }
};

// Plane z's contribution to the outputs that have it as their ez = +1 plane (kPrev:
// output z - k), their own plane (kCur: output z, with its stored seed) and their ez = -1
// plane (kNext: output z + k).  kSparse: skip the plane's arithmetic when every id it
// loaded is EMPTY on every lane of the wave.
template <int kRows, int kCols, bool kSparse, bool kInC, bool kPrev, bool kCur, bool kNext>
__device__ __forceinline__ void plane(const int32_t* __restrict__ in, uint32_t plane_elems, int32_t z, int32_t k,
                                      const Column<kInC>& c, int32_t& a_prev, int32_t& a_cur, int32_t& a_next)
{
    using S = Slots<kRows, kCols>;
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in, plane_elems, z);
    uint32_t v[9];  // complemented ids
#pragma unroll
    for (int q = 0; q < 9; ++q)
        if (S::has(q)) {
            const uint32_t raw = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)c.off[q], 0, 0);
            v[q] = kInC ? raw : ~(raw | (uint32_t)c.inv[q]);
        }
    if (kSparse) {
        uint32_t any = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (S::has(q)) any |= v[q];
        if (__builtin_amdgcn_readfirstlane((uint32_t)(__ballot(any != 0u) != 0ull)) == 0u) return;
    }
    const int32_t m_cur = key_factor(z), m_prev = key_factor(z - k), m_next = key_factor(z + k);
    int32_t kp[9], kc[9], kn[9];
    int32_t self = kNoKey;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        kp[q] = kc[q] = kn[q] = kNoKey;
        if (!S::has(q)) continue;
        Cand cd = prep(v[q], c.qxy, q);
        asm volatile("" : "+v"(cd.W));  // W once per seed; each key below is one multiply-add on it
        if (kPrev) kp[q] = cand_key(cd, m_prev);
        if (kCur) {
            if (q == 4) self = cand_key(cd, m_cur) - 5;  // the stored seed: rank 0 instead of 1 + 4
            else kc[q] = cand_key(cd, m_cur);
        }
        if (kNext) kn[q] = cand_key(cd, m_next);
    }
    if (kPrev) a_prev = min(a_prev, min9(kp) + 18);
    if (kCur) a_cur = min(a_cur, min(min9(kc) + 9, self));
    if (kNext) a_next = min(a_next, min9(kn));
}

// work-group `blk` (remapped task index) of a pass over one grid: positions
// [cb kThreads, (cb+1) kThreads) of the plane's columns in the pass's row order (x fastest,
// waves take consecutive positions across row ends, so no lane idles at the end of a row),
// z task bz; tab = rank_table(nx, ny, k)
template <int kCh, int kRows, int kCols, bool kSparse, bool kInC>
__device__ __forceinline__ void jfa_block(const int32_t* __restrict__ in, int32_t* __restrict__ out, int32_t nx,
                                          int32_t ny, int32_t nz, int32_t k, int64_t blk, const int32_t* tab,
                                          uint32_t omask)
{
    const uint32_t plane_elems = (uint32_t)nx * (uint32_t)ny;  // grids hold at most 2^30 points
    const int64_t gc = ceil_div(plane_elems, kThreads);
    const int64_t cb = blk % gc;
    const int32_t bz = (int32_t)(blk / gc);
    const int64_t pos = cb * kThreads + threadIdx.x;  // position in the pass's row order
    if (pos >= plane_elems) return;
    const int32_t i = (int32_t)(pos / nx), x = (int32_t)(pos - (int64_t)i * nx);
    const int32_t y = pass_row(i, nx, ny, k);
    const uint32_t col = (uint32_t)x + (uint32_t)nx * (uint32_t)y;  // element index within a plane

    Column<kInC> c;
    const uint32_t own = 4u * col;
#pragma unroll
    for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
        for (int ex = -1; ex <= 1; ++ex) {
            const int q = 3 * (ey + 1) + (ex + 1);
            const int32_t qx = x + ex * k, qy = y + ey * k;
            const bool ok = qx >= 0 && qx < nx && qy >= 0 && qy < ny;
            const uint32_t off = 4u * ((uint32_t)qx + (uint32_t)nx * (uint32_t)qy);  // bytes
            c.off[q] = ok ? off : (kInC ? kOutside : own);
            c.inv[q] = ok ? 0 : -1;
        }
    c.qxy = __builtin_bit_cast(short2_t, (1023u - (uint32_t)x) | ((1023u - (uint32_t)y) << 16));

    // the winner's id is reloaded from the query its rank names and stored complemented
    // (omask 0) or plain (omask all ones); real candidates have keys below 0 (d^2 <= 3 1023^2
    // against (4095 - pz)^2 >= 3072^2), EMPTY ones at least 0
    const uint32_t xmask = (kInC ? 0u : ~0u) ^ omask;
    auto emit = [&](int32_t pz, int32_t best) {
        const uint32_t p = col + plane_elems * (uint32_t)pz;
        uint32_t id = omask;
        if (best < 0) id = (uint32_t)in[(uint32_t)((int32_t)p + tab[best & 31])] ^ xmask;
        out[p] = (int32_t)id;
    };

    const ZTasks zt = z_tasks(nz, k, kCh);
    int32_t r0, r1, mlo, mhi;
    if (zt.per_res > 1) {
        r0 = bz / zt.per_res;
        r1 = r0 + 1;
        mlo = (bz - r0 * zt.per_res) * zt.len;
        mhi = mlo + zt.len;
    } else {
        r0 = bz;  // classes bz, bz + count, ... (stride rstep)
        r1 = zt.res;
        mlo = 0;
        mhi = 0x7FFFFFFF;
    }
    const int32_t rstep = zt.per_res > 1 ? 1 : zt.count;
#define RTSDF_PLANE(P, C, N, zz) \
    plane<kRows, kCols, kSparse, kInC, P, C, N>(in, plane_elems, zz, k, c, a_prev, a_cur, a_next)
    for (int32_t r = r0; r < r1; r += rstep) {
        const int32_t mcount = (nz - r + k - 1) / k;  // lattice points z = r + m k < nz
        const int32_t m0 = mlo, m1 = min(mhi, mcount);
        if (m0 >= m1) continue;
        // accumulators of outputs m - 1, m, m + 1 while plane m streams in
        int32_t a_prev = kNoKey, a_cur = kNoKey, a_next = kNoKey;
        if (m0 >= 1) {  // plane m0 - 1 is the ez = -1 plane of output m0
            RTSDF_PLANE(false, false, true, r + (m0 - 1) * k);
            a_cur = a_next;
            a_next = kNoKey;
        }
        for (int32_t m = m0; m < m1; ++m) {
            const int32_t z = r + m * k;
            const bool first = m == m0, last = m + 1 == m1;
            if (!first && !last) RTSDF_PLANE(true, true, true, z);
            else if (first && last) RTSDF_PLANE(false, true, false, z);
            else if (first) RTSDF_PLANE(false, true, true, z);
            else RTSDF_PLANE(true, true, false, z);
            if (!first) emit(z - k, a_prev);
            a_prev = a_cur;
            a_cur = a_next;
            a_next = kNoKey;
        }
        // plane m1 is the ez = +1 plane of the chain's last output
        if (m1 < mcount) RTSDF_PLANE(true, false, false, r + m1 * k);
        emit(r + (m1 - 1) * k, a_prev);
    }
#undef RTSDF_PLANE
}

// launch index -> task index: XCD x (= launch index mod 8) runs tasks [x per, (x+1) per)
__device__ inline int64_t xcd_task(uint32_t b, uint32_t nblocks)
{
    const uint32_t per = nblocks / kXcds;  // the launch is padded to a multiple of 8
    return (int64_t)(b % kXcds) * per + b / kXcds;
}

// kInC: the input holds complemented ids (every pass of a call but the first); omask: all
// ones when the output is to hold plain ids (the last pass), else 0
template <int kCh, int kRows, int kCols, bool kSparse, bool kInC>
__global__ __launch_bounds__(kThreads) void k_jfa_stream(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int32_t nx,
                                                          int32_t ny, int32_t nz, int32_t k, int64_t tasks,
                                                          uint32_t omask)
{
    const int64_t t = xcd_task(blockIdx.x, gridDim.x);
    if (t >= tasks) return;  // padding (whole work-group)
    __shared__ int32_t tab[32];
    rank_table(tab, nx, ny, k);
    __syncthreads();
    jfa_block<kCh, kRows, kCols, kSparse, kInC>(in, out, nx, ny, nz, k, t, tab, omask);
}

// work-groups of a pass over one grid before padding
__host__ __device__ inline int64_t pass_tasks(const rtsdf_grid& g, int32_t k, int32_t ch)
{
    return ceil_div((int64_t)g.nx * g.ny, kThreads) * z_tasks(g.nz, k, ch).count;
}

// One pass over every object still flooding: the task index picks the object from this
// pass's prefix table, then the object's own geometry and offset; object o reads the
// buffer holding its pass-p input (its start buffer alternates with p).
template <bool kSparse, bool kInC>
__global__ __launch_bounds__(kThreads) void k_jfa_batched(const char* __restrict__ plan, int32_t nobj,
                                                           int32_t pass, int32_t* __restrict__ seeds,
                                                           int32_t* __restrict__ scratch)
{
    const BatchView v = batch_view(plan, nobj);
    const int32_t* prefix = v.pass_prefix + (int64_t)pass * (nobj + 1);
    const int64_t b = xcd_task(blockIdx.x, gridDim.x);
    if (b >= prefix[nobj]) return;  // padding (whole work-group)
    const int32_t o = find_object(prefix, nobj, (int32_t)b);
    const BatchObject& ob = v.obj[o];
    const int32_t k = jfa_offset(ob.k0, ob.nhalf, pass);
    const int32_t nx = ob.g.nx, ny = ob.g.ny, nz = ob.g.nz;
    const bool from_scratch = (ob.flip ^ (pass & 1)) != 0;
    const int32_t* in = (from_scratch ? scratch : seeds) + ob.vox_off;
    int32_t* out = (from_scratch ? seeds : scratch) + ob.vox_off;
    __shared__ int32_t tab[32];
    rank_table(tab, nx, ny, k);
    __syncthreads();
    const uint32_t omask = pass + 1 == ob.nsteps ? ~0u : 0u;  // the object's last pass stores plain ids
    jfa_block<kChunk, 3, 3, kSparse, kInC>(in, out, nx, ny, nz, k, b - prefix[o], tab, omask);
}

unsigned padded(int64_t tasks) { return (unsigned)(ceil_div(tasks, kXcds) * kXcds); }

}  // namespace

int64_t jfa_pass_blocks(const rtsdf_grid& g, int32_t k) { return pass_tasks(g, k, kChunk); }

// pass p of an object's halving schedule has offset P / 2^(p+1), P the longest side n rounded
// up to a power of two (n <= P < 2n); for a power-of-two RTSDF_JFA_SPARSE = S, S x offset >= n
// then holds exactly for p < log2(S), the passes jfa_sparse picks for a single grid
constexpr int ilog2(int v) { return v > 1 ? 1 + ilog2(v / 2) : 0; }
constexpr int kSparsePasses = RTSDF_JFA_SPARSE > 0 ? ilog2(RTSDF_JFA_SPARSE) : 0;

hipError_t jfa_batched_pass(const BatchView& hv, const void* dplan, int32_t* seeds, int32_t* scratch, int32_t pass,
                            hipStream_t s)
{
    const int32_t blocks = hv.h->pass_blocks[pass];
    if (blocks == 0) return hipSuccess;
    // pass 0 reads the voxelized (plain) ids, later passes complemented ones
    const dim3 grid(padded(blocks)), block(kThreads);
    if constexpr (kSparsePasses > 0) {
        if (pass < kSparsePasses) {  // an object's offsets halve from half its longest side: as jfa_sparse
            if (pass == 0)
                hipLaunchKernelGGL((k_jfa_batched<true, false>), grid, block, 0, s, (const char*)dplan, hv.h->nobj,
                                   pass, seeds, scratch);
            else
                hipLaunchKernelGGL((k_jfa_batched<true, true>), grid, block, 0, s, (const char*)dplan, hv.h->nobj,
                                   pass, seeds, scratch);
            return hipGetLastError();
        }
    }
    if (pass == 0)
        hipLaunchKernelGGL((k_jfa_batched<false, false>), grid, block, 0, s, (const char*)dplan, hv.h->nobj, pass,
                           seeds, scratch);
    else
        hipLaunchKernelGGL((k_jfa_batched<false, true>), grid, block, 0, s, (const char*)dplan, hv.h->nobj, pass,
                           seeds, scratch);
    return hipGetLastError();
}

namespace {

template <int kCh, int kRows, int kCols, bool kSparse>
void launch_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, bool in_c, uint32_t omask,
                 int64_t tasks, hipStream_t s)
{
    const dim3 grid(padded(tasks)), block(kThreads);
    if (in_c)
        hipLaunchKernelGGL((k_jfa_stream<kCh, kRows, kCols, kSparse, true>), grid, block, 0, s, in, out, g.nx, g.ny,
                           g.nz, k, tasks, omask);
    else
        hipLaunchKernelGGL((k_jfa_stream<kCh, kRows, kCols, kSparse, false>), grid, block, 0, s, in, out, g.nx, g.ny,
                           g.nz, k, tasks, omask);
}

template <int kCh, int kRows, int kCols>
void launch_pass_sparse(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, bool sparse, bool in_c,
                        uint32_t omask, int64_t tasks, hipStream_t s)
{
    if constexpr (RTSDF_JFA_SPARSE > 0)
        if (sparse) return launch_pass<kCh, kRows, kCols, true>(in, out, g, k, in_c, omask, tasks, s);
    launch_pass<kCh, kRows, kCols, false>(in, out, g, k, in_c, omask, tasks, s);
}

template <int kCh>
void launch_pass_modes(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, bool sparse, bool in_c,
                       uint32_t omask, int64_t tasks, hipStream_t s)
{
    // neighbour rows (columns) at +-k lie outside the grid everywhere once k >= ny (nx)
    const bool rows1 = k >= g.ny, cols1 = k >= g.nx;
    if (rows1 && cols1) launch_pass_sparse<kCh, 1, 1>(in, out, g, k, sparse, in_c, omask, tasks, s);
    else if (rows1) launch_pass_sparse<kCh, 1, 3>(in, out, g, k, sparse, in_c, omask, tasks, s);
    else if (cols1) launch_pass_sparse<kCh, 3, 1>(in, out, g, k, sparse, in_c, omask, tasks, s);
    else launch_pass_sparse<kCh, 3, 3>(in, out, g, k, sparse, in_c, omask, tasks, s);
}

}  // namespace

bool jfa_sparse(const rtsdf_grid& g, int32_t k)
{
    return RTSDF_JFA_SPARSE > 0 && (int64_t)RTSDF_JFA_SPARSE * k >= std::max(g.nx, std::max(g.ny, g.nz));
}

hipError_t jfa_pass(const int32_t* in, int32_t* out, const rtsdf_grid& g, int32_t k, bool in_plain, bool out_plain,
                    hipStream_t s)
{
    const bool sparse = jfa_sparse(g, k);
    const bool few = pass_tasks(g, k, kChunk) < kFewBlocks;  // small grids: shorter chunks, more blocks
    const int64_t tasks = pass_tasks(g, k, few ? kChunkSmall : kChunk);
    const uint32_t omask = out_plain ? ~0u : 0u;
    if (few) launch_pass_modes<kChunkSmall>(in, out, g, k, sparse, !in_plain, omask, tasks, s);
    else launch_pass_modes<kChunk>(in, out, g, k, sparse, !in_plain, omask, tasks, s);
    return hipGetLastError();
}

}  // namespace rtsdf
