// Ray sampling of the masked grid points (section 2.1) against the software BVH.
//
// A persistent grid; each lane owns one work unit at a time -- a masked voxel and a group of
// its rays j (all x of them unless the mask is small, see below) -- and traces those rays
// one after the other, keeping the minimum distance, hit counts and argmin record in
// registers, and folds them into the voxel's accumulators once at the end (min / add are
// order-free, so the result does not depend on scheduling).  A lane whose ray ends starts
// its next ray at once, and a lane whose unit is done takes the next unit from its wave's
// chunk of the unit range (one cursor atomic per chunk of units: device-scope atomics on
// one address serialise across the chip), so divergent ray lengths neither idle lanes nor
// leave a tail of busy waves.  A mask with fewer than about two voxels per lane of the grid
// is split into groups of consecutive rays so that every lane has work.  The unit range is
// split into contiguous ranges, RTSDF_RAY_RANGES / 8 per XCD (work-groups are dealt to
// the 8 XCDs round-robin), each with its own cursor on its own cache line (device-scope
// atomics on one line serialise); a wave takes units from a range of its own XCD, so list
// reads and the hierarchy working set stay in that XCD's L2, and moves on to the next
// range -- its own XCD's first -- when that one is exhausted.
// The loop touches no cold memory: directions are drawn in registers and accumulators are
// updated with fire-and-forget atomics, because on CDNA loads retire in order and one
// HBM-latency load would stall every later node fetch of the wave.
// Each loop iteration does at most one node visit and one triangle test per lane.
//
// Traversal of the 4-wide hierarchy: the four child boxes are tested at once, the hits are
// sorted by entry distance (packed into uint keys with the slot in the two low bits, the
// distance rounded down, which can only keep more boxes), the nearest node is visited next
// and the others go on a per-lane stack of (child code, entry t) in LDS (t rounded down to
// its top 16 bits there, which can only keep more boxes) that spills to private memory past
// kLdsDepth.  Leaf ranges are tested one triangle per iteration; a lane holds up to two
// pending ranges, so that meeting a second leaf does not stop its traversal.  A box
// is culled only when its entry parameter exceeds the best hit so far (ties are still
// visited, because the tie-break is the triangle index).  Box tests may round freely:
// every triangle box is widened by 2*pad while a hit's computed point must lie within pad
// of its triangle's box, so a box holding a hit is never culled and the result equals the
// brute-force least (t, triangle index).
#include <mutex>

#include "traverse.h"
#include "tuning.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 256;
// waves per SIMD the register budget allows: single-object and batched instances (the
// latter keeps its object's grid and hierarchy per lane, and needs more registers)
template <bool kBatch>
constexpr int kMinWaves = kBatch ? RTSDF_RAY_WAVES_BATCH : RTSDF_RAY_WAVES;
constexpr int kPopTrips = RTSDF_RAY_POP_TRIPS;  // stack pops per lane and iteration (0: no limit)
// LDS stack entries per lane (6 bytes each: a child code and the top 16 bits of its entry
// t): the CU's 160 KB shared by kMinWaves waves on each of 4 SIMDs
template <bool kBatch>
constexpr int kLdsDepth = 163840 / (4 * kMinWaves<kBatch>) / (64 * 6);
static_assert(kLdsDepth<false> >= 4 && kLdsDepth<false> < kMaxStack, "stack depth");
static_assert(kLdsDepth<true> >= 4 && kLdsDepth<true> < kMaxStack, "stack depth");
constexpr int kXcds = 8;
constexpr int32_t kChunk = RTSDF_RAY_CHUNK;            // work units a wave takes per cursor atomic
constexpr int32_t kChunkSmall = RTSDF_RAY_CHUNK_SMALL;  // ... when there are few units per lane
constexpr int32_t kChunkRays = RTSDF_RAY_CHUNK_RAYS;   // ... and at least this many rays
constexpr int32_t kStartBatch = RTSDF_RAY_START_BATCH;  // idle lanes restarted together
constexpr int kRanges = RTSDF_RAY_RANGES;  // unit ranges, each with its own cursor
constexpr int kSub = kRanges / kXcds;      // ranges per XCD
constexpr int kCursorStride = 32;          // cursors are 128 bytes apart
static_assert(kSub * kXcds == kRanges, "ranges split evenly over the XCDs");
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

// cursors[r * kCursorStride] walks range r = [r*units/kRanges, (r+1)*units/kRanges) of the
// work units; ranges x*kSub ... x*kSub + kSub - 1 belong to XCD x
__global__ void k_cursor_reset(int32_t* cursors)
{
    if (threadIdx.x < kRanges) cursors[threadIdx.x * kCursorStride] = 0;
}

// kBatch: the mask list indexes concatenated grids; each voxel's object (binary search over
// the plan's voxel prefix) supplies its grid, its hierarchy and the counter's object word.
template <bool kBatch>
__global__ __launch_bounds__(kThreads, kMinWaves<kBatch>) void k_raysample(const char* __restrict__ bvh, const rtsdf_grid g,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ count_p, int32_t x,
                                                        uint32_t k0, uint32_t k1, uint32_t frame,
                                                        const uint32_t* __restrict__ frame_dev,
                                                        uint32_t obj, float* __restrict__ dmin,
                                                        uint32_t* __restrict__ hits,
                                                        uint64_t* __restrict__ argmin,
                                                        int32_t* __restrict__ cursors, const char* plan,
                                                        int32_t nobj)
{
    constexpr int kDepth = kLdsDepth<kBatch>;
    // The stack: child codes, and their entry t's top 16 bits (t rounded down, so that a pop
    // culls no box the exact t would keep); spilled entries keep the whole t.
    __shared__ int32_t s_code[kDepth][kThreads];
    __shared__ uint16_t s_t16[kDepth][kThreads];
    // spilled entries as one 64-bit word (t bits high): an array shaped like an LDS one lets
    // the compiler merge the two reads into one flat load, which occupies the vector-memory
    // path even for LDS addresses
    uint64_t p_key[kMaxStack - kDepth];

    // the hierarchy and grid of the current voxel (fixed for a single object)
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
    rtsdf_grid lg = g;
    uint32_t lobj = obj;
    if (!kBatch) use_bvh(bvh);
    const int32_t count = *count_p;
    // Work units: (listed voxel, group of consecutive rays).  A mask smaller than about two
    // units per lane of the grid is split into ray groups so that every lane has work;
    // otherwise a unit is a whole voxel.  units <= max(count, 2 * lanes) < 2^31.
    const int64_t lanes = (int64_t)gridDim.x * kThreads;
    int32_t ngroups = (int32_t)min((int64_t)x, max((int64_t)1, (2 * lanes) / max((int64_t)count, (int64_t)1)));
    const uint32_t gsize = (uint32_t)((x + ngroups - 1) / ngroups);
    ngroups = (int32_t)((x + (int32_t)gsize - 1) / (int32_t)gsize);
    const int32_t units = count * ngroups;
    // many units per lane: short chunks balance the tail; few: long chunks, fewer atomics;
    // and never fewer than kChunkRays rays per atomic (with one ray per unit the cursor
    // atomics, serialised per XCD, would otherwise bound the launch)
    const int32_t chunk = max((int64_t)units >= 8 * lanes ? kChunk : kChunkSmall,
                              (int32_t)((kChunkRays + gsize - 1) / gsize));
    const float inf = __int_as_float(0x7f800000);
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    if (frame_dev != nullptr) frame = *frame_dev;  // the frame index as of when the kernel runs
    const uint32_t code0 = frame * (uint32_t)x;
    // the range this wave takes units from: one of its own XCD's
    int rng = (int)(blockIdx.x % kXcds) * kSub + (int)((blockIdx.x / kXcds) % kSub);
    int tried = 0;                        // ranges found exhausted
    int32_t q_next = 0, q_end = 0;        // the wave's current chunk of the unit range

    int32_t vid = -1;
    uint32_t lvid = 0;  // the voxel's index within its own grid (counter word)
    uint32_t j = 0, jend = 0;  // the unit's current and end ray
    float acc_d = inf;
    uint32_t acc_h = 0;
    uint64_t acc_a = ~0ull;
    float3 o = make_float3(0.f, 0.f, 0.f);
    bool alive = true, active = false;
    float3 w = o, inv = o, oinv = o;
    NearPlanes np{true, true, true};
    float tb = inf;
    int32_t bid = kNone;
    bool bfr = false;
    int32_t node = -1;
    int32_t pfirst = 0, pcount = 0;  // pending leaf range
    int32_t pfirst2 = 0, pcount2 = 0;  // a second one (only while the first is pending)
    int sp = 0;

    auto put = [&](int at, const ChildKey& k) {
        s_code[at][tid] = k.code;
        s_t16[at][tid] = (uint16_t)(k.t >> 16);
    };
    // (sp < kMaxStack always holds: deeper hierarchies are not traversed; the test keeps
    // the private array in bounds regardless)
    auto push = [&](const ChildKey& k) {
        if (sp < kDepth) {
            put(sp, k);
        } else if (sp < kMaxStack) {
            p_key[sp - kDepth] = stack_word(k);
        }
        sp = min(sp + 1, kMaxStack);
    };

    while (true) {
        // Lanes whose ray ended wait until kStartBatch of them (or the whole wave) can be
        // retired, refilled and restarted together: that code is long (Philox, Marsaglia,
        // set-up) and a wave pays for it whenever any lane runs it.
        const int32_t idle = (int32_t)__popcll(__ballot(alive && !active));
        const bool batch = idle >= kStartBatch || __ballot(active) == 0ull;
        // retire a finished ray; fold a finished voxel into its accumulators
        bool need = false;
        if (batch && alive && !active) {
            if (vid >= 0) {
                if (bid != kNone) {
                    acc_d = fminf(acc_d, tb);
                    acc_h += bfr ? 1u : 65536u;
                    const uint64_t rec = ((uint64_t)__float_as_uint(tb) << 32) | (uint64_t)(code0 + j);
                    acc_a = rec < acc_a ? rec : acc_a;
                }
                if (++j == jend) {
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
        // wave-cooperative refill: lanes take units from the wave's current chunk; an empty
        // chunk is replaced by one atomic on this XCD's cursor, and an
        // exhausted range moves the wave on to the next XCD's range
        uint64_t needers = __ballot(need);
        while (needers && tried < kRanges) {
            if (q_next >= q_end) {
                const int32_t lo = (int32_t)(((int64_t)units * rng) / kRanges);
                const int32_t hi = (int32_t)(((int64_t)units * (rng + 1)) / kRanges);
                int32_t base = 0;
                if (lane == 0) base = atomicAdd(&cursors[rng * kCursorStride], chunk);
                base = __shfl(base, 0) + lo;
                if (base >= hi) {
                    rng = (rng + 1) % kRanges;  // the next range: the same XCD's first
                    ++tried;
                    continue;
                }
                q_next = base;
                q_end = min(base + chunk, hi);
            }
            const int32_t rank = (int32_t)__popcll(needers & lt_mask);
            const int32_t take = min((int32_t)__popcll(needers), q_end - q_next);
            if (need && rank < take) {
                const int32_t u = q_next + rank;
                const int32_t q = u / ngroups;
                vid = list[q];
                need = false;
                j = (uint32_t)(u - q * ngroups) * gsize;
                jend = min(j + gsize, (uint32_t)x);
                acc_d = inf;
                acc_h = 0u;
                acc_a = ~0ull;
                lvid = (uint32_t)vid;
                if (kBatch) {
                    const BatchView bv = batch_view(plan, nobj);
                    const int32_t oi = find_object(bv.vox_prefix, nobj, (int64_t)vid);
                    const BatchObject& ob = bv.obj[oi];
                    lvid = (uint32_t)(vid - ob.vox_off);
                    lg = ob.g;
                    lobj = (uint32_t)oi;
                    use_bvh(bvh + ob.bvh_off);
                }
                const uint32_t nx = (uint32_t)lg.nx, ny = (uint32_t)lg.ny;
                const uint32_t row = lvid / nx;
                const uint32_t i0 = lvid - row * nx, i1 = row % ny, i2 = row / ny;
                o = make_float3(lg.org[0] + lg.h * ((float)i0 + 0.5f), lg.org[1] + lg.h * ((float)i1 + 0.5f),
                                lg.org[2] + lg.h * ((float)i2 + 0.5f));
            }
            q_next += take;
            needers = __ballot(need);
        }
        if (need) alive = false;
        // start the next ray
        if (batch && alive && !active) {
            w = sphere_direction(k0, k1, lvid, frame, j, lobj);
            inv = make_float3(slab_rcp(w.x), slab_rcp(w.y), slab_rcp(w.z));
            oinv = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
            np = near_planes(inv);
            tb = inf;
            bid = kNone;
            sp = 0;
            node = -1;
            pcount = 0;
            pcount2 = 0;
            if (nt > 0) {
                if (root >= 0 && !deep) {
                    node = root;
                } else if (root >= 0) {
                    pfirst = 0;  // every triangle, in sorted order: the same closest hit
                    pcount = nt;
                } else {
                    pfirst = leaf_first(root);
                    pcount = leaf_count(root);
                }
                active = true;
            }
        }
        if (__ballot(alive) == 0ull) break;
        if (!active) continue;
        // at most one triangle test ...
        if (pcount > 0) {
            test_leaf(tris, pfirst, o, w, pad, tb, bid, bfr);
            ++pfirst;
            --pcount;
            if (pcount == 0) {
                pfirst = pfirst2;
                pcount = pcount2;
                pcount2 = 0;
            }
        }
        // ... and one node visit per iteration
        if (node >= 0) {
            ChildKey s0, s1, s2, s3;
            node_keys(fetch_node(nodes, (uint32_t)node), np, inv, oinv, tb, s0, s1, s2, s3);
            sort4(s0, s1, s2, s3);
            // entered boxes sort first, so they are a prefix: push the entered ones of s1..s3,
            // farthest first; with room in LDS all three slots are written unconditionally
            // (slots past the new top are dead) and only the top moves
            const int nv = (int)entered(s1) + (int)entered(s2) + (int)entered(s3);
            if (sp + 3 <= kDepth) {
                put(sp, nv == 3 ? s3 : (nv == 2 ? s2 : s1));
                put(sp + 1, nv == 3 ? s2 : s1);
                put(sp + 2, s1);
                sp += nv;
            } else {
                if (entered(s3)) push(s3);
                if (entered(s2)) push(s2);
                if (entered(s1)) push(s1);
            }
            node = -1;
            if (entered(s0)) {
                const int32_t c0 = s0.code;
                if (c0 >= 0) {
                    node = c0;
                } else if (pcount == 0) {
                    pfirst = leaf_first(c0);
                    pcount = leaf_count(c0);
                } else if (pcount2 == 0) {
                    pfirst2 = leaf_first(c0);
                    pcount2 = leaf_count(c0);
                } else {
                    push(s0);
                }
            }
        }
        // refill node / pending leaf from the stack
        int trips = 0;
        while (node < 0 && sp > 0 && (kPopTrips == 0 || trips++ < kPopTrips)) {
            const int top = sp - 1;
            uint32_t tbits;
            int32_t e;
            if (top < kDepth) {
                tbits = (uint32_t)s_t16[top][tid] << 16;
                e = s_code[top][tid];
            } else {
                const uint64_t w = p_key[top - kDepth];
                tbits = (uint32_t)(w >> 32);
                e = word_code(w);
            }
            if (__uint_as_float(tbits) > tb) {
                sp = top;
                continue;
            }
            if (e >= 0) {
                node = e;
                sp = top;
            } else if (pcount == 0) {
                pfirst = leaf_first(e);
                pcount = leaf_count(e);
                sp = top;
            } else if (pcount2 == 0) {
                pfirst2 = leaf_first(e);
                pcount2 = leaf_count(e);
                sp = top;
            } else {
                break;
            }
        }
        if (node < 0 && pcount == 0 && sp == 0) active = false;
    }
}

// Work cursors of the allocation-free entry point: one array per GPU, held until the
// process ends and shared by every call on that GPU.  Host code never passes this name to
// a kernel (on the host it is only a stand-in for the symbol): it uses the device address
// that scratch_ptr() looks up.
constexpr size_t kScratchBytes = 4096;
static_assert(sizeof(int32_t) * kRanges * kCursorStride <= kScratchBytes, "cursors fit the static scratch");
static __device__ __align__(256) int32_t scratch[kScratchBytes / sizeof(int32_t)];

}  // namespace

size_t raysample_work_bytes(int64_t, int32_t) { return sizeof(int32_t) * kRanges * kCursorStride; }

size_t raysample_scratch_bytes() { return kScratchBytes; }

hipError_t raysample_scratch(void** out)
{
    // the array's address on each device, looked up once per device with that device current
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list, const int32_t* count,
                     int64_t capacity, int32_t x, uint64_t key, uint32_t frame, const uint32_t* frame_dev,
                     uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    int32_t* cursors = (int32_t*)work;
    hipLaunchKernelGGL(k_cursor_reset, dim3(1), dim3(kRanges), 0, s, cursors);
    // exactly the resident grid: more groups would only start after others finish
    static int resident = 0;
    if (resident == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raysample<false>, kThreads, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        resident = per_cu * cus;
    }
    const int64_t want = ceil_div(capacity, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(kXcds, std::min<int64_t>(want, resident));
    hipLaunchKernelGGL(k_raysample<false>, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g, list, count, x,
                       (uint32_t)key, (uint32_t)(key >> 32), frame, frame_dev, obj, dmin, hits, argmin, cursors,
                       nullptr, 0);
    return hipGetLastError();
}

hipError_t raysample_batched(const BatchView& hv, const void* dplan, const void* bvh, const int32_t* list,
                             const int32_t* count, int64_t capacity, int32_t x, uint64_t key, uint32_t frame,
                             float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    int32_t* cursors = (int32_t*)work;
    hipLaunchKernelGGL(k_cursor_reset, dim3(1), dim3(kRanges), 0, s, cursors);
    static int resident = 0;
    if (resident == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raysample<true>, kThreads, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        resident = per_cu * cus;
    }
    const int64_t want = ceil_div(capacity, kThreads);
    const unsigned groups = (unsigned)std::max<int64_t>(kXcds, std::min<int64_t>(want, resident));
    const rtsdf_grid g0 = hv.obj[0].g;  // unused in batch mode
    hipLaunchKernelGGL(k_raysample<true>, dim3(groups), dim3(kThreads), 0, s, (const char*)bvh, g0, list, count, x,
                       (uint32_t)key, (uint32_t)(key >> 32), frame, nullptr, 0u, dmin, hits, argmin, cursors,
                       (const char*)dplan, hv.h->nobj);
    return hipGetLastError();
}

}  // namespace rtsdf
