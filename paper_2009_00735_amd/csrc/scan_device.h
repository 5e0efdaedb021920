// Device-wide exclusive prefix sum, hand-written for the ROI query and the
// adaptive ROI grid:  out[i] = in[0] + ... + in[i-1] for i = 0 .. n (so
// out[0] = 0 and out[n] is the total).  Three launches on the caller's
// stream, all deterministic (fixed summation order):
//   1. k_scan_tiles   one workgroup per tile of kScanTile inputs: the tile sum;
//   2. k_scan_carry   one workgroup: exclusive scan of the tile sums in place,
//                     and out[n] = the total;
//   3. k_scan_apply   one workgroup per tile: the scan inside the tile plus the
//                     tile's carry.
// IN and OUT may differ in width (e.g. int32 counts into int64 offsets); the
// sums are formed in OUT.
#pragma once

#include "ar_internal.h"

namespace ar {
namespace scan {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;   // 4096 inputs per workgroup

inline int64_t tiles(int64_t n) { return (n + kTile - 1) / kTile; }

// Block-wide exclusive scan of one value per thread (Hillis-Steele in LDS);
// returns this thread's exclusive prefix and the block total in *sum.
template <typename T> __device__ __forceinline__ T block_exclusive(T v, T *sh, T *sum)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const T t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : T(0);
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    *sum = sh[kThreads - 1];
    const T incl = sh[threadIdx.x];
    __syncthreads();
    return incl - v;
}

template <typename IN, typename OUT>
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const IN *__restrict__ in, int64_t n, OUT *__restrict__ tsum)
{
    __shared__ OUT sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPerThread;
    OUT s = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k)
        if (base + k < n) s += (OUT)in[base + k];
    OUT total;
    block_exclusive<OUT>(s, sh, &total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

template <typename OUT>
__global__ __launch_bounds__(kThreads) void k_scan_carry(OUT *__restrict__ tsum, int64_t n_tiles, OUT *__restrict__ out_n)
{
    __shared__ OUT sh[kThreads];
    OUT carry = 0;
    for (int64_t c0 = 0; c0 < n_tiles; c0 += kThreads) {
        const int64_t i = c0 + threadIdx.x;
        const OUT v = i < n_tiles ? tsum[i] : OUT(0);
        OUT total;
        const OUT ex = block_exclusive<OUT>(v, sh, &total);
        if (i < n_tiles) tsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *out_n = carry;
}

template <typename IN, typename OUT>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const IN *__restrict__ in, int64_t n,
                                                         const OUT *__restrict__ tsum, OUT *__restrict__ out)
{
    __shared__ OUT sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPerThread;
    OUT v[kPerThread];
    OUT s = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        v[k] = base + k < n ? (OUT)in[base + k] : OUT(0);
        s += v[k];
    }
    OUT total;
    OUT run = block_exclusive<OUT>(s, sh, &total) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// Queue the exclusive scan of n >= 0 inputs into out[0 .. n]; `tsum` is
// device workspace of at least tiles(n) OUT values (may be NULL for n = 0).
template <typename IN, typename OUT>
ar_status exclusive_scan(const IN *in, int64_t n, OUT *out, OUT *tsum, hipStream_t s)
{
    const int64_t nt = tiles(n);
    if (nt > 0) {
        k_scan_tiles<IN, OUT><<<(unsigned)nt, kThreads, 0, s>>>(in, n, tsum);
        AR_HIP(hipGetLastError());
    }
    k_scan_carry<OUT><<<1, kThreads, 0, s>>>(tsum, nt, out + n);
    AR_HIP(hipGetLastError());
    if (nt > 0) {
        k_scan_apply<IN, OUT><<<(unsigned)nt, kThreads, 0, s>>>(in, n, tsum, out);
        AR_HIP(hipGetLastError());
    }
    return AR_OK;
}

}  // namespace scan
}  // namespace ar
