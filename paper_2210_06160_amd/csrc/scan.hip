// Device-wide exclusive prefix sums: reduce per block, scan the block sums (recursively),
// then scan each block again adding its offset.  Used for triangle candidate offsets,
// ray-mask compaction and radix-sort digit offsets.
#include "internal.h"

namespace rtsdf {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // items per block

template <typename T>
__device__ T block_exclusive_scan(T v, T* lds_wave, T* block_total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    T inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) lds_wave[wave] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) {
        T s = lds_wave[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    *block_total = tot;
    return off + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_reduce(const T* __restrict__ in, int64_t n,
                                                      T* __restrict__ sums)
{
    __shared__ T lds[kThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) acc += in[base + i];
    T total;
    block_exclusive_scan<T>(acc, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan(const T* in, T* out, int64_t n,
                                                    const T* __restrict__ offsets,
                                                    T* __restrict__ total_out)
{
    __shared__ T lds[kThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    T v[kItems];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        acc += v[i];
    }
    T total;
    T run = block_exclusive_scan<T>(acc, lds, &total) + (offsets ? offsets[blockIdx.x] : T(0));
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) *total_out = run;
}

template <typename T>
size_t scan_work_elems(int64_t n)
{
    size_t e = 0;
    int64_t m = n;
    while (m > kTile) {
        m = ceil_div(m, kTile);
        e += (size_t)m;
        e = (e + 63) & ~size_t(63);
    }
    return e;
}

template <typename T>
hipError_t scan_impl(const T* in, T* out, int64_t n, T* total, T* work, hipStream_t s)
{
    if (n <= 0) {
        if (total) {
            // write a zero total with a one-thread scan of nothing
            hipLaunchKernelGGL((k_scan<T>), dim3(1), dim3(kThreads), 0, s, in, out, (int64_t)0,
                               (const T*)nullptr, total);
        }
        return hipGetLastError();
    }
    const int64_t nb = ceil_div(n, kTile);
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan<T>), dim3(1), dim3(kThreads), 0, s, in, out, n,
                           (const T*)nullptr, total);
        return hipGetLastError();
    }
    T* sums = work;
    T* rest = work + ((nb + 63) & ~int64_t(63));
    hipLaunchKernelGGL((k_reduce<T>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, sums);
    hipError_t e = scan_impl<T>(sums, sums, nb, (T*)nullptr, rest, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan<T>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n,
                       (const T*)sums, total);
    return hipGetLastError();
}

}  // namespace

size_t scan_work_bytes_u32(int64_t n) { return align256(scan_work_elems<uint32_t>(n) * 4 + 256); }
size_t scan_work_bytes_u64(int64_t n) { return align256(scan_work_elems<uint64_t>(n) * 8 + 256); }

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                              void* work, hipStream_t s)
{
    return scan_impl<uint32_t>(in, out, n, total, (uint32_t*)work, s);
}

hipError_t scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                              void* work, hipStream_t s)
{
    return scan_impl<uint64_t>(in, out, n, total, (uint64_t*)work, s);
}

int persistent_groups(int threads_per_group)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    const int waves = threads_per_group / kWave;
    return cus * (32 / (waves > 0 ? waves : 1));
}

}  // namespace rtsdf
