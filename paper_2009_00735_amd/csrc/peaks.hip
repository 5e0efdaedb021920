// Measured peak rates of the units the kernels are bound by (the roofline
// denominators): HBM copy, LDS 16-byte reads, conflict-free LDS atomics,
// non-packed FP32 FMA, the transcendental unit (alone and issued beside FMA
// work), BF16 and FP32 MFMA, and random 8-byte LDS reads.  Each probe runs a fixed loop on a grid of eight
// workgroups per compute unit and is timed with HIP events around the launch.

#include "ar_internal.h"

namespace ar {
namespace peaks {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kBlock = 256;

// Grid-stride float4 copy (measured faster here than four loads in flight
// per thread).
__global__ __launch_bounds__(kBlock) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 16-byte LDS reads, 64 consecutive float4 per wavefront instruction (no bank
// conflicts); four adds per read keep the loads alive.
__global__ __launch_bounds__(kBlock) void k_lds_read(int iters, float *__restrict__ out)
{
    __shared__ float4 buf[1024];
    for (int i = threadIdx.x; i < 1024; i += kBlock) buf[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int it = 0; it < iters; ++it) {
        const float4 v = buf[(threadIdx.x + it * 64) & 1023];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

// LDS integer atomics without return, every lane on its own bank.
__global__ __launch_bounds__(kBlock) void k_lds_atomic(int iters, unsigned *__restrict__ out)
{
    __shared__ unsigned h[1024];
    for (int i = threadIdx.x; i < 1024; i += kBlock) h[i] = 0u;
    __syncthreads();
    for (int it = 0; it < iters; ++it) atomicAdd(&h[(threadIdx.x + it * kBlock) & 1023], 1u);
    __syncthreads();
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = h[threadIdx.x];
}

// NF independent FMA chains and NS independent v_sin_f32 chains per lane,
// four iterations per loop trip so loop control is a small share of the issue.
template <int NF, int NS>
__global__ __launch_bounds__(kBlock) void k_alu(int iters, float b, float c, float *__restrict__ out)
{
    float a[NF > 0 ? NF : 1], s[NS > 0 ? NS : 1];
#pragma unroll
    for (int k = 0; k < NF; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int it = 0; it < iters; it += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int k = 0; k < NF; ++k) a[k] = fmaf(a[k], b, c);
#pragma unroll
            for (int k = 0; k < NS; ++k) s[k] = __builtin_amdgcn_sinf(s[k]);
        }
    }
    float r = 0.f;
#pragma unroll
    for (int k = 0; k < NF; ++k) r += a[k];
#pragma unroll
    for (int k = 0; k < NS; ++k) r += s[k];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = r;
}

// 8-byte LDS reads at pseudo-random addresses: a per-lane linear congruential
// sequence picks one of 8192 entries (64 KB) per read, so a wavefront's reads
// collide on banks as random look-ups do.
__global__ __launch_bounds__(kBlock) void k_lds_gather(int iters, float *__restrict__ out)
{
    __shared__ uint2 buf[8192];
    for (int i = threadIdx.x; i < 8192; i += kBlock) buf[i] = make_uint2(i, 3 * i);
    __syncthreads();
    uint32_t h = threadIdx.x * 2654435761u + blockIdx.x * 40503u + 1u;
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
        h = h * 1664525u + 1013904223u;
        const uint2 v = buf[h >> 19];
        acc += v.x ^ v.y;
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = (float)acc;
}

// v_mfma_f32_32x32x16_bf16 on four independent accumulators per wavefront.
__global__ __launch_bounds__(kBlock) void k_mfma(int iters, float *__restrict__ out)
{
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(0.001f * (float)(threadIdx.x + i));
        b[i] = (__bf16)(0.002f * (float)(threadIdx.x - i));
    }
    f32x16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
    }
    float r = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) r += acc[j][i];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = r;
}

// v_mfma_f32_32x32x2_f32 on four independent accumulators per wavefront.
__global__ __launch_bounds__(kBlock) void k_mfma_f32(int iters, float *__restrict__ out)
{
    const float a = 0.001f * (float)threadIdx.x, b = 0.002f * (float)(threadIdx.x + 1);
    f32x16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
    }
    float r = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) r += acc[j][i];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = r;
}

}  // namespace peaks
}  // namespace ar

namespace {

// Time one launch (after one warm-up launch) in seconds.
template <typename Launch> ar_status time_launch(Launch launch, double *seconds)
{
    hipEvent_t e0, e1;
    AR_HIP(hipEventCreate(&e0));
    AR_HIP(hipEventCreate(&e1));
    launch();
    AR_HIP(hipGetLastError());
    AR_HIP(hipEventRecord(e0, nullptr));
    launch();
    AR_HIP(hipEventRecord(e1, nullptr));
    AR_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    AR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *seconds = ms * 1e-3;
    return AR_OK;
}

}  // namespace

extern "C" {

ar_status ar_measure_peaks(ar_context *ctx, double *out, int32_t n_out)
{
    using namespace ar::peaks;
    AR_CHECK(ctx != nullptr && out != nullptr, "ctx/out is NULL");
    AR_CHECK(n_out >= AR_PEAK_COUNT, "out must hold %d values", (int)AR_PEAK_COUNT);
    AR_HIP(hipSetDevice(ctx->device));
    const int blocks = ctx->cu_count * 8;
    const size_t threads = (size_t)blocks * kBlock;
    ar::DeviceBuffer sink;
    AR_TRY(sink.reserve(threads * sizeof(float)));
    double t = 0.0;

    // HBM: 1 GiB read + 1 GiB written
    {
        const size_t n = (size_t)1 << 26;   // 1 GiB of float4
        ar::DeviceBuffer a, b;
        AR_TRY(a.reserve(n * sizeof(float4)));
        AR_TRY(b.reserve(n * sizeof(float4)));
        AR_HIP(hipMemset(a.ptr, 0, n * sizeof(float4)));
        AR_TRY(time_launch([&] { k_copy<<<blocks, kBlock>>>(a.as<float4>(), b.as<float4>(), n); }, &t));
        out[AR_PEAK_HBM_BYTES] = 2.0 * (double)(n * sizeof(float4)) / t;
    }
    const int it_lds = 8192, it_alu = 4096, it_mfma = 1024;
    AR_TRY(time_launch([&] { k_lds_read<<<blocks, kBlock>>>(it_lds, sink.as<float>()); }, &t));
    out[AR_PEAK_LDS_BYTES] = (double)threads * it_lds * 16.0 / t;
    AR_TRY(time_launch([&] { k_lds_atomic<<<blocks, kBlock>>>(it_lds, sink.as<unsigned>()); }, &t));
    out[AR_PEAK_LDS_ATOMICS] = (double)threads * it_lds / t;
    double t_fma = 0.0;
    AR_TRY(time_launch([&] { k_alu<16, 0><<<blocks, kBlock>>>(it_alu, 0.999f, 1e-3f, sink.as<float>()); }, &t_fma));
    out[AR_PEAK_FP32_FMA_FLOPS] = (double)threads * it_alu * 16.0 * 2.0 / t_fma;
    AR_TRY(time_launch([&] { k_alu<0, 16><<<blocks, kBlock>>>(it_alu, 0.999f, 1e-3f, sink.as<float>()); }, &t));
    out[AR_PEAK_SIN] = (double)threads * it_alu * 16.0 / t;
    // 16 FMA chains beside 4 sin chains: equal to the FMA-only time if the
    // transcendental unit runs beside the FMA pipeline
    AR_TRY(time_launch([&] { k_alu<16, 4><<<blocks, kBlock>>>(it_alu, 0.999f, 1e-3f, sink.as<float>()); }, &t));
    out[AR_PEAK_SIN_OVERLAP] = t_fma / t;
    AR_TRY(time_launch([&] { k_mfma<<<blocks, kBlock>>>(it_mfma, sink.as<float>()); }, &t));
    out[AR_PEAK_BF16_MFMA_FLOPS] = (double)blocks * (kBlock / 64) * it_mfma * 4.0 * (32.0 * 32.0 * 16.0 * 2.0) / t;
    AR_TRY(time_launch([&] { k_mfma_f32<<<blocks, kBlock>>>(it_mfma / 4, sink.as<float>()); }, &t));
    out[AR_PEAK_FP32_MFMA_FLOPS] = (double)blocks * (kBlock / 64) * (it_mfma / 4) * 4.0 * (32.0 * 32.0 * 2.0 * 2.0) / t;
    AR_TRY(time_launch([&] { k_lds_gather<<<blocks, kBlock>>>(it_lds, sink.as<float>()); }, &t));
    out[AR_PEAK_LDS_GATHER8] = (double)threads * it_lds / t;
    return AR_OK;
}

}  // extern "C"
