// VALU issue-rate probe: a known number of vector ALU instructions of one kind per lane, so
// that the lane-operations per second an integer- or float-bound kernel can reach on this
// chip are measured rather than assumed, instruction by instruction, and so that the
// SQ_INSTS_VALU counter can be checked against an exact instruction count.
//
// Each thread runs `iters` trips of a block of 16 instructions of one kind, written in
// inline assembly so that the compiler can neither fold nor reorder them.  In the
// independent forms the 16 instructions rotate over 8 accumulators (two per accumulator
// per trip, so up to 8 are in flight per wave); in the dependent forms every instruction
// reads the previous one's result.  Only VALU operations appear in the assembly (no memory
// access); the result is stored only when it equals a value it cannot reach in practice,
// which keeps the chains live without adding memory traffic.  Operand values are
// arbitrary bit patterns: the issue rate of these instructions does not depend on them.
//
// Built into its own library (libvalupeak.so); the path does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kPerTrip = 16;

#define TWO(x) x x
#define OUTS8(a) "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7])

// The operand shapes: dst = op(dst, b[, c]) over 8 accumulators (twice each per trip).
#define I2(ins)                                                                                         \
    asm volatile(TWO(ins " %0, %0, %8\n\t" ins " %1, %1, %8\n\t" ins " %2, %2, %8\n\t" ins " %3, %3, %8\n\t" ins \
                     " %4, %4, %8\n\t" ins " %5, %5, %8\n\t" ins " %6, %6, %8\n\t" ins " %7, %7, %8\n\t")            \
                 : OUTS8(a)                                                                             \
                 : "v"(b))
#define I3(ins)                                                                                         \
    asm volatile(TWO(ins " %0, %0, %8, %9\n\t" ins " %1, %1, %8, %9\n\t" ins " %2, %2, %8, %9\n\t" ins          \
                     " %3, %3, %8, %9\n\t" ins " %4, %4, %8, %9\n\t" ins " %5, %5, %8, %9\n\t" ins " %6, %6, %8, %9\n\t" \
                     ins " %7, %7, %8, %9\n\t")                                                          \
                 : OUTS8(a)                                                                             \
                 : "v"(b), "v"(c))
// dst += op(b, c) (the accumulating VOP2 forms)
#define IACC(ins)                                                                                       \
    asm volatile(TWO(ins " %0, %8, %9\n\t" ins " %1, %8, %9\n\t" ins " %2, %8, %9\n\t" ins " %3, %8, %9\n\t" ins \
                     " %4, %8, %9\n\t" ins " %5, %8, %9\n\t" ins " %6, %8, %9\n\t" ins " %7, %8, %9\n\t")            \
                 : OUTS8(a)                                                                             \
                 : "v"(b), "v"(c))
// v_cndmask reads vcc (whatever it holds)
#define ICND(ins)                                                                                       \
    asm volatile(TWO(ins " %0, %0, %8, vcc\n\t" ins " %1, %1, %8, vcc\n\t" ins " %2, %2, %8, vcc\n\t" ins       \
                     " %3, %3, %8, vcc\n\t" ins " %4, %4, %8, vcc\n\t" ins " %5, %5, %8, vcc\n\t" ins             \
                     " %6, %6, %8, vcc\n\t" ins " %7, %7, %8, vcc\n\t")                                  \
                 : OUTS8(a)                                                                             \
                 : "v"(b))
// v_cmp writing vcc, then v_cndmask reading it: 8 of each per trip
#define ICMPSEL(ins)                                                                                    \
    asm volatile(TWO("v_cmp_lt_u32 vcc, %0, %8\n\t" ins " %1, %1, %8, vcc\n\t"                               \
                     "v_cmp_lt_u32 vcc, %2, %8\n\t" ins " %3, %3, %8, vcc\n\t"                               \
                     "v_cmp_lt_u32 vcc, %4, %8\n\t" ins " %5, %5, %8, vcc\n\t"                               \
                     "v_cmp_lt_u32 vcc, %6, %8\n\t" ins " %7, %7, %8, vcc\n\t")                              \
                 : OUTS8(a)                                                                             \
                 : "v"(b)                                                                               \
                 : "vcc")
// v_cndmask_b32 (VOP3 form) with a mask in an SGPR pair other than vcc
#define ICNDS(ins)                                                                                      \
    asm volatile(TWO(ins " %0, %0, %8, %9\n\t" ins " %1, %1, %8, %9\n\t" ins " %2, %2, %8, %9\n\t" ins          \
                     " %3, %3, %8, %9\n\t" ins " %4, %4, %8, %9\n\t" ins " %5, %5, %8, %9\n\t" ins " %6, %6, %8, %9\n\t" \
                     ins " %7, %7, %8, %9\n\t")                                                          \
                 : OUTS8(a)                                                                             \
                 : "v"(b), "s"(m))
// dst = op(dst)
#define INOT(ins)                                                                                       \
    asm volatile(TWO(ins " %0, %0\n\t" ins " %1, %1\n\t" ins " %2, %2\n\t" ins " %3, %3\n\t" ins " %4, %4\n\t" ins \
                     " %5, %5\n\t" ins " %6, %6\n\t" ins " %7, %7\n\t")                               \
                 : OUTS8(a))
// v_mad_u64_u32 dst64 = src0 * src1 + src2_64 (the 32 x 32 -> 64 products of Philox): 8
// independent 64-bit accumulators would need 16 registers, so 4 are rotated twice per trip
#define IMAD64(ins)                                                                                     \
    asm volatile(TWO(TWO(ins " %0, s[0:1], %4, %5, %0\n\t" ins " %1, s[0:1], %4, %5, %1\n\t" ins           \
                         " %2, s[0:1], %4, %5, %2\n\t" ins " %3, s[0:1], %4, %5, %3\n\t"))              \
                 : "+v"(w64[0]), "+v"(w64[1]), "+v"(w64[2]), "+v"(w64[3])                            \
                 : "v"(b), "v"(c)                                                                      \
                 : "s0", "s1")
// one chain: every instruction reads the previous result
#define D2(ins) asm volatile(TWO(TWO(TWO(TWO(ins " %0, %0, %1\n\t")))) : "+v"(a[0]) : "v"(b))
#define D3(ins) asm volatile(TWO(TWO(TWO(TWO(ins " %0, %0, %1, %2\n\t")))) : "+v"(a[0]) : "v"(b), "v"(c))

// (index, name, shape): the probe table
#define PROBES(X)                                  \
    X(0, "v_add_u32", I2)                          \
    X(1, "v_add_u32", D2)                          \
    X(2, "v_mad_u32_u24", I3)                      \
    X(3, "v_mad_u32_u24", D3)                      \
    X(4, "v_min3_i32", I3)                         \
    X(5, "v_dot2_i32_i16", I3)                     \
    X(6, "v_fma_f32", I3)                          \
    X(7, "v_lshl_or_b32", I3)                      \
    X(8, "v_sub_u32", I2)                          \
    X(9, "v_and_b32", I2)                          \
    X(10, "v_or_b32", I2)                          \
    X(11, "v_xor_b32", I2)                         \
    X(12, "v_lshlrev_b32", I2)                     \
    X(13, "v_lshrrev_b32", I2)                     \
    X(14, "v_min_i32", I2)                         \
    X(15, "v_max_u32", I2)                         \
    X(16, "v_mul_u32_u24", I2)                     \
    X(17, "v_mul_i32_i24", I2)                     \
    X(18, "v_mul_lo_u32", I2)                      \
    X(19, "v_add_f32", I2)                         \
    X(20, "v_mul_f32", I2)                         \
    X(21, "v_min_f32", I2)                         \
    X(22, "v_max_f32", I2)                         \
    X(23, "v_pk_add_u16", I2)                      \
    X(24, "v_pk_sub_i16", I2)                      \
    X(25, "v_pk_min_i16", I2)                      \
    X(26, "v_pk_lshlrev_b16", I2)                  \
    X(27, "v_pk_mul_lo_u16", I2)                   \
    X(28, "v_cndmask_b32", ICND)                   \
    X(29, "v_mad_i32_i24", I3)                     \
    X(30, "v_max3_i32", I3)                        \
    X(31, "v_med3_i32", I3)                        \
    X(32, "v_min3_f32", I3)                        \
    X(33, "v_add3_u32", I3)                        \
    X(34, "v_and_or_b32", I3)                      \
    X(35, "v_or3_b32", I3)                         \
    X(36, "v_lshl_add_u32", I3)                    \
    X(37, "v_add_lshl_u32", I3)                    \
    X(38, "v_bfe_u32", I3)                         \
    X(39, "v_bfi_b32", I3)                         \
    X(40, "v_perm_b32", I3)                        \
    X(41, "v_dot2_u32_u16", I3)                    \
    X(42, "v_pk_mad_i16", I3)                      \
    X(43, "v_sad_u32", I3)                         \
    X(44, "v_alignbit_b32", I3)                    \
    X(45, "v_xad_u32", I3)                         \
    X(46, "v_dot2c_i32_i16", IACC)                 \
    X(47, "v_fmac_f32", IACC)                      \
    X(48, "v_dot4c_i32_i8", IACC)                  \
    X(49, "v_pk_fma_f16", I3)                      \
    X(50, "v_max3_f32", I3)                        \
    X(51, "v_med3_f32", I3)                        \
    X(52, "v_fma_f32", D3)                         \
    X(53, "v_min_i32", D2)                         \
    X(54, "v_mul_u32_u24", D2)                     \
    X(55, "v_cndmask_b32", ICMPSEL)                \
    X(56, "v_cndmask_b32_e64", ICNDS)              \
    X(57, "v_not_b32", INOT)                       \
    X(58, "v_cvt_f32_u32", INOT)                   \
    X(59, "v_mov_b32", INOT)                       \
    X(60, "v_cvt_f32_ubyte0", INOT)                \
    X(61, "v_mul_hi_u32", I2)                      \
    X(62, "v_mad_u64_u32", IMAD64)

#define COUNT(i, n, s) +1
constexpr int kOps = 0 PROBES(COUNT);

template <int kOp>
struct Probe;
#define DEF(i, n, s)                                                                                     \
    template <>                                                                                          \
    struct Probe<i> {                                                                                    \
        __device__ static inline void run(uint32_t (&a)[8], uint64_t (&w64)[4], uint32_t b, uint32_t c, \
                                          uint64_t m)                                                 \
        {                                                                                              \
            s(n);                                                                                      \
        }                                                                                              \
    };
PROBES(DEF)

template <int kOp>
__global__ __launch_bounds__(256) void k_valu(uint32_t* __restrict__ sink, int32_t iters, uint32_t seed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = seed ^ (t * 2654435761u + (uint32_t)i);
    const uint32_t b = (seed * 3u + 1u) | 1u, c = seed >> 3;
    const uint64_t m = 0x5555555555555555ull ^ (uint64_t)seed;  // a lane mask in SGPRs
    uint64_t w64[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w64[i] = ((uint64_t)a[2 * i] << 32) | a[2 * i + 1];
    for (int32_t i = 0; i < iters; ++i) Probe<kOp>::run(a, w64, b, c, m);
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r ^= a[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) r ^= (uint32_t)w64[i] ^ (uint32_t)(w64[i] >> 32);
    if (r == 0x9E3779B9u) sink[t & 255u] = r;
}

#define NAME(i, n, s) n,
#define SHAPE(i, n, s) #s,
const char* const kNames[] = {PROBES(NAME)};
const char* const kShapes[] = {PROBES(SHAPE)};

}  // namespace

extern "C" {

// Number of probe kinds, and VALU instructions each thread issues per trip.
int valu_peak_ops(void) { return kOps; }
int valu_peak_per_trip(void) { return kPerTrip; }
// Instruction mnemonic of probe `op`, and its form: I2 / I3 (dst = op(dst, b[, c]), 8
// independent chains), INOT (dst = op(dst)), IACC (dst += op(b, c)), ICND (v_cndmask on
// vcc), ICMPSEL (v_cmp_lt_u32 into vcc then the op reading it, 8 of each per trip), ICNDS
// (v_cndmask on a mask in another SGPR pair), IMAD64 (64-bit accumulators), D2 / D3 (one
// dependent chain).  NULL for an unknown op.
const char* valu_peak_name(int32_t op) { return op >= 0 && op < kOps ? kNames[op] : nullptr; }
const char* valu_peak_shape(int32_t op) { return op >= 0 && op < kOps ? kShapes[op] : nullptr; }

// Enqueues one probe of kind `op` on `stream`: `blocks` work-groups of 256 threads, `iters`
// trips each, so iters * 16 instructions of that kind are issued per lane.  `sink` is a
// device buffer of at least 256 uint32 (written only on an unreachable result).  Returns 0,
// or -1 for bad arguments, or -4 when the launch fails.
int valu_peak_launch(int32_t op, int32_t blocks, int32_t iters, uint32_t seed, uint32_t* sink, void* stream)
{
    if (blocks < 1 || iters < 1 || sink == nullptr) return -1;
    hipStream_t s = (hipStream_t)stream;
    switch (op) {
#define CASE(i, n, sh)                                                                                   \
    case i: hipLaunchKernelGGL(k_valu<i>, dim3((unsigned)blocks), dim3(256), 0, s, sink, iters, seed); break;
        PROBES(CASE)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
