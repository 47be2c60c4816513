// Ray sampling of the masked grid points (section 2.1) against the software BVH.
//
// A persistent grid.  Each wave walks a stream of rays (listed voxel, ray j < x), voxel by
// voxel, and keeps a pool of the next 64 of them in registers, one per lane: the whole wave
// fills the pool at once (the voxel's centre and the ray's direction from the counter-based
// generator, each lane one ray), and a lane whose ray ends takes the next pooled ray with a
// few cross-lane reads, so restarts are cheap enough to run for a handful of idle lanes and
// the generator runs with every lane busy.  A voxel's results (least hit distance, front and
// back hit counts, least (t, ray) record) are collected in a slot in LDS with LDS atomics
// while its rays are traced and folded into the global accumulators with one set of atomics
// when the slot is reused or the wave ends (min / add are order-free, so the result does not
// depend on scheduling); a ray that outlives its voxel's slot adds its own result to the
// global accumulators.  Waves take voxels in chunks (one cursor atomic per chunk: device-scope
// atomics on one address serialise across the chip).  The voxel range is split into
// contiguous ranges, RTSDF_RAY_RANGES / 8 per XCD (work-groups are dealt to the 8 XCDs
// round-robin), each with its own cursor on its own cache line (device-scope atomics on one
// line serialise); a wave takes chunks from a range of its own XCD, so list reads and the
// hierarchy working set stay in that XCD's L2, and moves on to the next range -- its own
// XCD's first -- when that one is exhausted.
// The loop touches no cold memory: directions are drawn in registers and accumulators are
// updated in LDS or with fire-and-forget atomics, because on CDNA loads retire in order and
// one HBM-latency load would stall every later node fetch of the wave.
// Each loop iteration does at most RTSDF_RAY_VISITS node visits per lane, with a triangle
// test after every second one.
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
constexpr int kWaves = kThreads / kWave;  // waves per work-group
// waves per SIMD the register budget allows: single-object and batched instances (the
// latter keeps its object's hierarchy per lane, and needs more registers)
template <bool kBatch>
constexpr int kMinWaves = kBatch ? RTSDF_RAY_WAVES_BATCH : RTSDF_RAY_WAVES;
constexpr int kPopTrips = RTSDF_RAY_POP_TRIPS;  // stack pops per lane and node visit (0: no limit)
constexpr int kVisits = RTSDF_RAY_VISITS;  // node visits per lane and loop iteration
static_assert(kVisits >= 1, "at least one node visit per iteration");
// the rounds (node visit, stack pops) that a triangle test precedes: every second one from
// the second on (the first, with one round per iteration)
__device__ constexpr bool test_before(int round) { return kVisits > 1 ? round % 2 == 1 : round == 0; }

// A voxel's results while its rays are traced (one slot per voxel in a per-wave ring).
struct alignas(16) VoxelSlot {
    int32_t vid;       // listed voxel (-1: none)
    float ox, oy, oz;  // its centre
    uint32_t d;        // bits of the least hit distance (positive floats order as integers)
    uint32_t h;        // front hits | back hits << 16
    uint64_t a;        // least (t bits, ray code) record
};
constexpr int kSlots = RTSDF_RAY_SLOTS;  // slots per wave (a power of two)
static_assert((kSlots & (kSlots - 1)) == 0 && kSlots >= 2 && kSlots <= 128, "slots: a power of two <= 128");
// voxels one pool fill gives a slot: at most half the ring, so that a fill never takes over
// a slot whose voxel still has pooled rays; the fill's later voxels (few rays per voxel)
// have none, and their rays add their results to the global accumulators themselves
constexpr int kFillVoxels = kSlots / 2;
constexpr uint32_t kNoSlot = 0xFFu;
// rays per voxel from which a fill of 64 rays needs no more than kFillVoxels voxels; with
// fewer, the kernel instance whose fills give the surplus voxels no slot runs instead
constexpr int32_t kFewRays = kWave / kFillVoxels;
template <bool kBatch>
constexpr int kSlotBytes = kWaves * kSlots * (int)(sizeof(VoxelSlot) + (kBatch ? sizeof(int32_t) : 0));
// LDS stack entries per lane (6 bytes each: a child code and the top 16 bits of its entry
// t): what the work-group's slots leave of its share of the CU's 160 KB (kMinWaves
// work-groups of 4 waves per CU), the share rounded down to whole KiB (LDS behaves as if
// allocated in KiB granules: a work-group of 27,136 bytes, within its 27,306-byte share but
// not a whole number of KiB, ran as if one work-group fewer fitted per CU)
template <bool kBatch>
constexpr int kGroupLds = (163840 / kMinWaves<kBatch>) / 1024 * 1024;
template <bool kBatch>
constexpr int kLdsDepth = (kGroupLds<kBatch> - kSlotBytes<kBatch>) / (kThreads * 6);
static_assert(kLdsDepth<false> >= 4 && kLdsDepth<false> < kMaxStack, "stack depth");
static_assert(kLdsDepth<true> >= 4 && kLdsDepth<true> < kMaxStack, "stack depth");
constexpr int kXcds = 8;
constexpr int32_t kChunk = RTSDF_RAY_CHUNK;            // voxels a wave takes per cursor atomic (at most)
constexpr int32_t kStartBatch = RTSDF_RAY_START_BATCH;  // idle lanes restarted together
constexpr int kRanges = RTSDF_RAY_RANGES;  // voxel ranges, each with its own cursor
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

// cursors[r * kCursorStride] walks range r = [r*count/kRanges, (r+1)*count/kRanges) of the
// listed voxels; ranges x*kSub ... x*kSub + kSub - 1 belong to XCD x
__global__ void k_cursor_reset(int32_t* cursors)
{
    if (threadIdx.x < kRanges) cursors[threadIdx.x * kCursorStride] = 0;
}

// kBatch: the mask list indexes concatenated grids; each voxel's object (binary search over
// the plan's voxel prefix) supplies its grid, its hierarchy and the counter's object word.
// kFew (x < 8): a fill of 64 rays spans more voxels than it has slots for; the later ones
// go without a slot (their rays add to the global accumulators themselves), and the pool
// holds each ray's voxel.  With x >= 8 a fill spans at most kFillVoxels voxels.
template <bool kBatch, bool kFew>
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
    __shared__ VoxelSlot s_slot[kWaves][kSlots];
    __shared__ int32_t s_obj[kWaves][kBatch ? kSlots : 1];  // a slot's object (batched)
    // spilled entries as one 64-bit word (t bits high): an array shaped like an LDS one lets
    // the compiler merge the two reads into one flat load, which occupies the vector-memory
    // path even for LDS addresses
    uint64_t p_key[kMaxStack - kDepth];

    // the hierarchy of the current ray's object (fixed for a single object)
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
    if (!kBatch) use_bvh(bvh);
    int32_t cur_obj = -1;  // the object whose hierarchy is loaded (batched)
    const int32_t count = *count_p;
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wv = tid / kWave;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    // Voxels per pool fill (whole voxels while x <= 64), and per cursor atomic: about a
    // quarter of each wave's share, within [one fill, kChunk].
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    const int32_t fill_vox = kFew ? max(1, kWave / x) : min(kFillVoxels, max(1, kWave / x));
    const int32_t chunk = (int32_t)max((int64_t)fill_vox, min((int64_t)kChunk, (int64_t)count / (4 * nwaves)));
    const float inf = __int_as_float(0x7f800000);
    if (frame_dev != nullptr) frame = *frame_dev;  // the frame index as of when the kernel runs
    const uint32_t code0 = frame * (uint32_t)x;
    VoxelSlot* const slots = s_slot[wv];
    if (lane < kSlots) slots[lane].vid = -1;

    auto flush = [&](int32_t v, uint32_t d, uint32_t h, uint64_t a) {
        atomicMin((uint32_t*)&dmin[v], d);
        atomicAdd(&hits[v], h);
        if (argmin) atomicMin((unsigned long long*)&argmin[v], (unsigned long long)a);
    };
    // the centre of voxel lvid of grid lg
    auto centre = [](const rtsdf_grid& lg, uint32_t lvid) {
        const uint32_t nx = (uint32_t)lg.nx, ny = (uint32_t)lg.ny;
        const uint32_t row = lvid / nx;
        const uint32_t i0 = lvid - row * nx, i1 = row % ny, i2 = row / ny;
        return make_float3(lg.org[0] + lg.h * ((float)i0 + 0.5f), lg.org[1] + lg.h * ((float)i1 + 0.5f),
                           lg.org[2] + lg.h * ((float)i2 + 0.5f));
    };
    // a batched voxel's object, its grid and its index there
    auto locate = [&](int32_t vid, rtsdf_grid& lg, uint32_t& lvid) {
        const BatchView bv = batch_view(plan, nobj);
        const int32_t oi = find_object(bv.vox_prefix, nobj, (int64_t)vid);
        const BatchObject& ob = bv.obj[oi];
        lvid = (uint32_t)(vid - ob.vox_off);
        lg = ob.g;
        return oi;
    };

    // the ray stream (wave-uniform): next ray j_next of listed voxel v_next, in the chunk
    // [v_next, v_end) of range rng
    int rng = (int)(blockIdx.x % kXcds) * kSub + (int)((blockIdx.x / kXcds) % kSub);
    int tried = 0;  // ranges found exhausted
    int32_t v_next = 0, v_end = 0;
    uint32_t j_next = 0;
    uint32_t slot_next = 0;        // the slot the next voxel takes (mod kSlots)
    uint32_t slot_cont = kNoSlot;  // (kFew) the slot of the voxel the last fill left unfinished
    int32_t pool_n = 0, pool_at = 0;  // pooled rays, and the next one to hand out
    bool more = true;              // the stream may still hold rays
    float3 pw = make_float3(0.f, 0.f, 0.f);  // this lane's pooled ray: direction,
    uint32_t pmeta = 0;                      // slot | ray j << 8,
    int32_t pvid = 0;                        // and (kFew) voxel

    // Fills the pool with the stream's next rays (lane i takes ray i); returns their number
    // (0: the stream is exhausted).  Wave-uniform control flow.
    auto fill = [&]() -> int32_t {
        while (v_next >= v_end && tried < kRanges) {
            const int32_t lo = (int32_t)(((int64_t)count * rng) / kRanges);
            const int32_t hi = (int32_t)(((int64_t)count * (rng + 1)) / kRanges);
            int32_t base = 0;
            if (lane == 0) base = atomicAdd(&cursors[rng * kCursorStride], chunk);
            base = __builtin_amdgcn_readfirstlane(__shfl(base, 0)) + lo;  // wave-uniform
            if (base >= hi) {
                rng = (rng + 1) % kRanges;  // the next range: the same XCD's first
                ++tried;
                continue;
            }
            v_next = base;
            j_next = 0;
            v_end = min(base + chunk, hi);
        }
        if (v_next >= v_end) return 0;
        const uint32_t t = j_next + (uint32_t)lane;
        const uint32_t dv = t / (uint32_t)x;
        const uint32_t jj = t - dv * (uint32_t)x;
        const int32_t q = v_next + (int32_t)dv;
        const bool cont = j_next > 0u;  // the first voxel continues from the last fill
        bool valid;
        uint32_t sl;
        if constexpr (kFew) {
            // the fill's k-th new voxel takes slot slot_next + k while k < kFillVoxels
            valid = q < v_end;
            const uint32_t k = dv - (cont ? 1u : 0u);
            sl = (cont && dv == 0u) ? slot_cont
                                    : (k < (uint32_t)kFillVoxels ? (slot_next + k) & (uint32_t)(kSlots - 1) : kNoSlot);
        } else {
            valid = q < v_end && (int32_t)dv < kFillVoxels;
            sl = (slot_next - (cont ? 1u : 0u) + dv) & (uint32_t)(kSlots - 1);
        }
        if (valid) {
            const int32_t vid = list[q];
            uint32_t lvid = (uint32_t)vid, lobj = obj;
            rtsdf_grid lg = g;
            if (kBatch) lobj = (uint32_t)locate(vid, lg, lvid);
            pw = sphere_direction(k0, k1, lvid, frame, jj, lobj);
            pmeta = sl | (jj << 8);
            if (kFew) pvid = vid;
            if (jj == 0u && (!kFew || sl != kNoSlot)) {
                // the voxel's first ray: fold the slot's previous voxel into the global
                // accumulators and take the slot over
                VoxelSlot& s = slots[sl];
                const int32_t ov = s.vid;
                if (ov >= 0 && s.h != 0u) flush(ov, s.d, s.h, s.a);
                const uint32_t nx = (uint32_t)lg.nx, ny = (uint32_t)lg.ny;
                const uint32_t row = lvid / nx;
                const uint32_t i0 = lvid - row * nx, i1 = row % ny, i2 = row / ny;
                s.vid = vid;
                s.ox = lg.org[0] + lg.h * ((float)i0 + 0.5f);
                s.oy = lg.org[1] + lg.h * ((float)i1 + 0.5f);
                s.oz = lg.org[2] + lg.h * ((float)i2 + 0.5f);
                s.d = __float_as_uint(inf);
                s.h = 0u;
                s.a = ~0ull;
                if (kBatch) s_obj[wv][sl] = (int32_t)lobj;
            }
        }
        const int32_t n = (int32_t)__popcll(__ballot(valid));
        const uint32_t started = (uint32_t)__popcll(__ballot(valid && jj == 0u));
        if constexpr (kFew) {
            // the last pooled ray's slot carries over when its voxel has rays left
            slot_cont = (uint32_t)__shfl((int32_t)sl, n - 1);
            slot_next = (slot_next + min(started, (uint32_t)kFillVoxels)) & (uint32_t)(kSlots - 1);
        } else {
            slot_next = (slot_next + started) & (uint32_t)(kSlots - 1);
        }
        const uint32_t tn = j_next + (uint32_t)n;
        const uint32_t dn = tn / (uint32_t)x;
        v_next += (int32_t)dn;
        j_next = tn - dn * (uint32_t)x;
        return n;
    };

    // the current ray
    int32_t vid = -1;  // its voxel
    uint32_t slot = 0, j = 0;
    bool active = false, has_ray = false;  // tracing; holding a result not yet collected
    float3 o = make_float3(0.f, 0.f, 0.f);
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
        // Idle lanes are restarted together once kStartBatch of them (or the whole wave) wait.
        const uint64_t act = __ballot(active);
        const bool batch = (more && (int32_t)__popcll(~act) >= kStartBatch) || act == 0ull;
        if (batch) {
            // collect the finished rays into their voxels' slots
            if (has_ray && !active) {
                has_ray = false;
                if (bid != kNone) {
                    const uint32_t hv = bfr ? 1u : 65536u;
                    const uint64_t rec = ((uint64_t)__float_as_uint(tb) << 32) | (uint64_t)(code0 + j);
                    VoxelSlot& s = slots[kFew ? slot & (uint32_t)(kSlots - 1) : slot];
                    if ((!kFew || slot != kNoSlot) && s.vid == vid) {
                        atomicMin(&s.d, __float_as_uint(tb));
                        atomicAdd(&s.h, hv);
                        atomicMin((unsigned long long*)&s.a, (unsigned long long)rec);
                    } else {
                        flush(vid, __float_as_uint(tb), hv, rec);  // no slot, or it has moved on
                    }
                }
            }
            // hand the pooled rays out to the idle lanes, refilling the pool as it empties
            bool need = !active && more;
            uint64_t needers = __ballot(need);
            while (needers) {
                if (pool_at >= pool_n) {
                    pool_n = fill();
                    pool_at = 0;
                    if (pool_n == 0) {
                        more = false;
                        break;
                    }
                }
                const int32_t k = pool_at + (int32_t)__popcll(needers & lt_mask);
                const bool take = need && k < pool_n;
                const int src = take ? k : lane;
                const float wx = __shfl(pw.x, src), wy = __shfl(pw.y, src), wz = __shfl(pw.z, src);
                const uint32_t meta = (uint32_t)__shfl((int32_t)pmeta, src);
                const int32_t mvid = kFew ? __shfl(pvid, src) : 0;
                if (take) {
                    need = false;
                    slot = meta & 0xFFu;
                    j = meta >> 8;
                    int32_t oi = 0;
                    if (!kFew || slot != kNoSlot) {
                        const int4 sv = *(const int4*)&slots[slot];  // vid, centre
                        vid = sv.x;
                        o = make_float3(__int_as_float(sv.y), __int_as_float(sv.z), __int_as_float(sv.w));
                        if (kBatch) oi = s_obj[wv][slot];
                    } else {
                        // a voxel without a slot: its centre from its index
                        vid = mvid;
                        uint32_t lvid = (uint32_t)vid;
                        rtsdf_grid lg = g;
                        if (kBatch) oi = locate(vid, lg, lvid);
                        o = centre(lg, lvid);
                    }
                    if (kBatch && oi != cur_obj) {
                        cur_obj = oi;
                        use_bvh(bvh + batch_view(plan, nobj).obj[oi].bvh_off);
                    }
                    w = make_float3(wx, wy, wz);
                    inv = make_float3(slab_rcp(w.x), slab_rcp(w.y), slab_rcp(w.z));
                    oinv = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
                    np = near_planes(inv);
                    tb = inf;
                    bid = kNone;
                    sp = 0;
                    node = -1;
                    pcount = 0;
                    pcount2 = 0;
                    has_ray = true;
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
                pool_at = min(pool_n, pool_at + (int32_t)__popcll(needers));
                needers = __ballot(need);
            }
        }
        if (!more && __ballot(active) == 0ull) break;
        if (!active) continue;
        // kVisits rounds of (node visit, stack pops) per iteration, with a triangle test after
        // every second visit: visits outnumber triangle tests about two to one per ray, and the
        // iteration's fixed costs (restart check, loop control) are paid once per kVisits visits
#pragma unroll
        for (int round = 0; round < kVisits; ++round) {
            if (test_before(round)) {
                // a triangle test
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
            }
            // a node visit ...
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
            // ... and at most kPopTrips stack pops to refill the node or a pending leaf range
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
        }
        if (node < 0 && pcount == 0 && sp == 0) active = false;
    }
    // fold the voxels still in the slots into the global accumulators (every ray of the
    // wave has been collected)
    if (lane < kSlots) {
        const VoxelSlot s = slots[lane];
        if (s.vid >= 0 && s.h != 0u) flush(s.vid, s.d, s.h, s.a);
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

// Work-groups of a launch: one lane per ray up to exactly the resident grid (more groups
// would only start after others finish).
template <bool kBatch, bool kFew>
unsigned ray_groups(int64_t capacity, int32_t x)
{
    static int resident = 0;
    if (resident == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_raysample<kBatch, kFew>, kThreads, 0) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        resident = per_cu * cus;
    }
    const int64_t want = ceil_div(capacity * (int64_t)x, kThreads);
    return (unsigned)std::max<int64_t>(kXcds, std::min<int64_t>(want, resident));
}

template <bool kBatch, bool kFew>
void launch_raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list, const int32_t* count,
                      int64_t capacity, int32_t x, uint64_t key, uint32_t frame, const uint32_t* frame_dev,
                      uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin, int32_t* cursors,
                      const void* plan, int32_t nobj, hipStream_t s)
{
    hipLaunchKernelGGL((k_raysample<kBatch, kFew>), dim3(ray_groups<kBatch, kFew>(capacity, x)), dim3(kThreads), 0,
                       s, (const char*)bvh, g, list, count, x, (uint32_t)key, (uint32_t)(key >> 32), frame,
                       frame_dev, obj, dmin, hits, argmin, cursors, (const char*)plan, nobj);
}

hipError_t raysample(const void* bvh, const rtsdf_grid& g, const int32_t* list, const int32_t* count,
                     int64_t capacity, int32_t x, uint64_t key, uint32_t frame, const uint32_t* frame_dev,
                     uint32_t obj, float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    int32_t* cursors = (int32_t*)work;
    hipLaunchKernelGGL(k_cursor_reset, dim3(1), dim3(kRanges), 0, s, cursors);
    if (x < kFewRays)
        launch_raysample<false, true>(bvh, g, list, count, capacity, x, key, frame, frame_dev, obj, dmin, hits,
                                      argmin, cursors, nullptr, 0, s);
    else
        launch_raysample<false, false>(bvh, g, list, count, capacity, x, key, frame, frame_dev, obj, dmin, hits,
                                       argmin, cursors, nullptr, 0, s);
    return hipGetLastError();
}

hipError_t raysample_batched(const BatchView& hv, const void* dplan, const void* bvh, const int32_t* list,
                             const int32_t* count, int64_t capacity, int32_t x, uint64_t key, uint32_t frame,
                             float* dmin, uint32_t* hits, uint64_t* argmin, void* work, hipStream_t s)
{
    if (capacity <= 0) return hipSuccess;
    int32_t* cursors = (int32_t*)work;
    hipLaunchKernelGGL(k_cursor_reset, dim3(1), dim3(kRanges), 0, s, cursors);
    const rtsdf_grid g0 = hv.obj[0].g;  // unused in batch mode
    if (x < kFewRays)
        launch_raysample<true, true>(bvh, g0, list, count, capacity, x, key, frame, nullptr, 0u, dmin, hits, argmin,
                                     cursors, dplan, hv.h->nobj, s);
    else
        launch_raysample<true, false>(bvh, g0, list, count, capacity, x, key, frame, nullptr, 0u, dmin, hits, argmin,
                                      cursors, dplan, hv.h->nobj, s);
    return hipGetLastError();
}

}  // namespace rtsdf
