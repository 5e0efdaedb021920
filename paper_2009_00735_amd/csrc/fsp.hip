// Reciprocal-space signatures on a cubic grid (Sec. 2.2, FSP paragraph,
// Eq. (2); supplement, reciprocal-space cost O(N_roi N_w L_D^3)):
//   amp[r][a][b][c] = |F(k)|,  F(k) = sum_w exp(-2 pi i k . d_w),
//   k = ((a - L/2), (b - L/2), (c - L/2)) dk,  dk = 2 k_max / L.
//
// The exponential factorises per axis, so each ROI is one complex GEMM
//   F[a][(b,c)] = sum_w X[a][w] B[w][(b,c)],
//   X[a][w] = exp(-2 pi i k_a x_w),  B[w][(b,c)] = exp(-2 pi i (k_b y_w + k_c z_w)),
// with M = L rows, N = L^2 columns and K = N_w atoms, evaluated on FP32
// MFMA (v_mfma_f32_32x32x2_f32, two atoms per instruction).  A wavefront owns
// 2 x 2 complex 32 x 32 output tiles and builds its operands in registers:
// per step, lane l forms X for rows l % 32 (+32) and B for columns l % 32
// (+32) of atom l / 32 (phases in turns, reduced to [-1/2, 1/2], then
// v_cos/v_sin), and 16 MFMAs accumulate Re F = Xr Br - Xi Bi and
// Im F = Xr Bi + Xi Br.  The 4 wavefronts of a workgroup share the row tiles
// and take 4 column blocks; the ROI's atoms pass through LDS in chunks.  Per
// pair of atoms a wavefront issues 16 MFMAs (32768 MACs) against 8
// transcendentals per lane, so the kernel is bound by the FP32 matrix rate.
#include <math.h>

#include "ar_internal.h"

namespace ar {
namespace fsp {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;
constexpr int kChunk = 512;   // atoms per LDS stage

// A wavefront owns TM x TN complex 32 x 32 tiles (TM row tiles, TN column
// tiles): per step its lanes form TM X entries and TN B entries, which feed
// 4 TM TN MFMAs.  grid: n_roi * row_blocks * col_blocks workgroups of 256
// threads; a workgroup covers 32 TM rows and 4 * 32 TN columns.
template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_fsp(const float4 *__restrict__ rel, const int64_t *__restrict__ offsets,
                                             int L, float dk, int row_blocks, int col_blocks,
                                             float *__restrict__ amp)
{
    __shared__ float4 xs[kChunk];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t b = blockIdx.x;
    const int cb = (int)(b % col_blocks);
    b /= col_blocks;
    const int rb = (int)(b % row_blocks);
    const int64_t r = b / row_blocks;

    const int half = L >> 1;
    const int row0 = rb * 32 * TM;                               // first row of the wave's tiles
    const int col0 = (cb * kWaves + wave) * 32 * TN;             // first column of the wave's tiles
    float ka[TM], kb[TN], kc[TN];
#pragma unroll
    for (int m = 0; m < TM; ++m) ka[m] = (float)(row0 + 32 * m + (lane & 31) - half) * dk;
#pragma unroll
    for (int n = 0; n < TN; ++n) {
        const int col = col0 + 32 * n + (lane & 31);
        const int bi = col / L, ci = col - bi * L;
        kb[n] = (float)(bi - half) * dk;
        kc[n] = (float)(ci - half) * dk;
    }
    const int kslot = lane >> 5;                                 // which of the step's two atoms

    f32x16 re[TM][TN], im[TM][TN];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int n = 0; n < TN; ++n)
#pragma unroll
            for (int i = 0; i < 16; ++i) re[m][n][i] = im[m][n][i] = 0.0f;

    const int64_t o0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - o0);
    for (int c0 = 0; c0 < nw; c0 += kChunk) {
        const int cnt = min(kChunk, nw - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += 256) xs[i] = rel[o0 + c0 + i];
        __syncthreads();
        for (int j = 0; j < cnt; j += 2) {
            const int w = j + kslot;
            const bool ok = w < cnt;
            const float4 x = xs[ok ? w : cnt - 1];
            // exp(-2 pi i t) = cos(2 pi t) - i sin(2 pi t), phases in turns;
            // the tail atom's X entries are zero
            float xr[TM], xi[TM], br[TN], bim[TN];
#pragma unroll
            for (int m = 0; m < TM; ++m) {
                float t = ka[m] * x.x;
                t -= rintf(t);
                xr[m] = ok ? __builtin_amdgcn_cosf(t) : 0.0f;
                xi[m] = ok ? -__builtin_amdgcn_sinf(t) : 0.0f;
            }
#pragma unroll
            for (int n = 0; n < TN; ++n) {
                float t = fmaf(kc[n], x.z, kb[n] * x.y);
                t -= rintf(t);
                br[n] = __builtin_amdgcn_cosf(t);
                bim[n] = -__builtin_amdgcn_sinf(t);
            }
#pragma unroll
            for (int m = 0; m < TM; ++m)
#pragma unroll
                for (int n = 0; n < TN; ++n) {
                    re[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[m], br[n], re[m][n], 0, 0, 0);
                    im[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[m], bim[n], im[m][n], 0, 0, 0);
                    re[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(-xi[m], bim[n], re[m][n], 0, 0, 0);
                    im[m][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(xi[m], br[n], im[m][n], 0, 0, 0);
                }
        }
    }
    // C layout of a 32x32 MFMA: lane l, value i -> row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
    const size_t L2 = (size_t)L * L;
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int n = 0; n < TN; ++n) {
            float *out = amp + (size_t)r * L * L2 + (size_t)(col0 + 32 * n + (lane & 31));
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int a = row0 + 32 * m + 8 * (i >> 2) + 4 * kslot + (i & 3);
                out[(size_t)a * L2] = sqrtf(fmaf(re[m][n][i], re[m][n][i], im[m][n][i] * im[m][n][i]));
            }
        }
}

template <int TM, int TN>
ar_status launch(const float *rel, const int64_t *offsets, int64_t n_roi, int L, float dk, float *amp,
                 hipStream_t s)
{
    const int row_blocks = L / (32 * TM);
    const int col_blocks = L * L / (32 * TN * kWaves);
    const int64_t blocks = n_roi * row_blocks * (int64_t)col_blocks;
    AR_CHECK(blocks < (int64_t)INT32_MAX, "too many workgroups (%lld): index fewer ROIs per call", (long long)blocks);
    k_fsp<TM, TN><<<(unsigned)blocks, 256, 0, s>>>((const float4 *)rel, offsets, L, dk, row_blocks, col_blocks, amp);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // namespace fsp
}  // namespace ar

extern "C" {

ar_status ar_fsp_amplitudes(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi, int32_t L,
                            float k_max, float *amp, void *stream)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(rel && offsets && amp, "rel/offsets/amp must not be NULL");
    AR_CHECK(n_roi >= 1, "n_roi must be >= 1");
    AR_CHECK(L >= 32 && L <= 512 && L % 32 == 0, "L must be a multiple of 32 in [32, 512], got %d", L);
    AR_CHECK(k_max > 0.0f && isfinite(k_max), "k_max must be finite and > 0");
    AR_HIP(hipSetDevice(ctx->device));
    const float dk = (float)(2.0 * (double)k_max / (double)L);
    hipStream_t s = (hipStream_t)stream;
    // 2 x 2 tiles per wavefront; L = 32 (or an odd multiple of 32) has a single row tile
    if (L % 64 == 0) return ar::fsp::launch<2, 2>(rel, offsets, n_roi, L, dk, amp, s);
    return ar::fsp::launch<1, 2>(rel, offsets, n_roi, L, dk, amp, s);
}

}  // extern "C"
