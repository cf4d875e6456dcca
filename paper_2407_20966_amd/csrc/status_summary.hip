// Per-bit counts of a status array, reduced on the device.
//
// Each wave counts its 64 words one bit at a time with a ballot and a
// population count, so the running counts are wave-uniform; lane b then holds
// the count of bit b, the waves of a workgroup combine theirs in LDS, and one
// 64-bit atomic add per bit and workgroup lands in the caller's counts.
// Integer sums: the result does not depend on the order of the adds.
#include "kbl_internal.h"

namespace kbl {
namespace {

constexpr int kStatusBits = 32;
constexpr int kStatusThreads = 256;

__global__ __launch_bounds__(64) void status_clear(uint64_t* counts) {
    if (threadIdx.x < kStatusBits) counts[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kStatusThreads) void status_count(const uint32_t* __restrict__ st,
                                                               int64_t n, uint64_t* counts) {
    __shared__ unsigned long long part[kStatusBits];
    if (threadIdx.x < kStatusBits) part[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    uint64_t mine = 0;   // lane b < 32: count of bit b over this wave's words
    for (int64_t i0 = (int64_t)blockIdx.x * kStatusThreads + (threadIdx.x & ~63); i0 < n;
         i0 += (int64_t)gridDim.x * kStatusThreads) {
        const int64_t i = i0 + lane;
        const uint32_t w = i < n ? st[i] : 0u;
#pragma unroll
        for (int b = 0; b < kStatusBits; ++b) {
            const uint64_t c = (uint64_t)__popcll(__ballot((w >> b) & 1u));
            if (lane == b) mine += c;
        }
    }
    if (lane < kStatusBits && mine) atomicAdd(&part[lane], (unsigned long long)mine);
    __syncthreads();
    if (threadIdx.x < kStatusBits && part[threadIdx.x])
        atomicAdd((unsigned long long*)&counts[threadIdx.x], part[threadIdx.x]);
}

}  // namespace

hipError_t launch_status_summary(const uint32_t* st, int64_t n, uint64_t* counts,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(status_clear, dim3(1), dim3(64), 0, stream, counts);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || n == 0) return err;
    int64_t blocks = (n + kStatusThreads - 1) / kStatusThreads;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(status_count, dim3((unsigned)blocks), dim3(kStatusThreads), 0, stream, st,
                       n, counts);
    return hipGetLastError();
}

}  // namespace kbl
