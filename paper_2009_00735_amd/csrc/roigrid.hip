// Adaptive ROI-grid refinement (Sec. 3.5, aluminium bicrystal; supplement,
// local grid refinement): scan with a coarse ROI grid, keep the ROIs whose
// peak intensity in a selected window reaches kappa times the best coarse
// ROI's, and split each kept ROI's grid cell into s^3 cells whose centres are
// the next ROIs.  The intensity of ROI r in window w is the per-atom peak
// amplitude I = max_v img[r][w][v] / N_r (0 for an empty ROI).
//
//   1. k_intensity   one workgroup per ROI: per-window maxima over the
//                    directions, divided by the atom count (FP32).
//   2. k_best        per window, the maximum over all ROIs.
//   3. k_keep        flag[r] = any selected window with I >= kappa * best.
//   4. exclusive scan of the flags (scan_device.h; one host read of the
//                    total).
//   5. k_emit        s^3 centres per kept ROI, in the order (kept ROI, x, y,
//                    z); each offset h (2i + 1 - s) / (2s) is evaluated in
//                    FP64 on the host, rounded to FP32 and added in FP32.
#include <math.h>

#include "ar_internal.h"
#include "scan_device.h"

namespace ar {
namespace roigrid {

constexpr int kMaxWin = 32;
constexpr int kMaxSplit = 16;

struct Offsets {
    float d[kMaxSplit];
};

__global__ __launch_bounds__(256) void k_intensity(const float *__restrict__ img, const int32_t *__restrict__ counts,
                                                   int n_win, int n_dir, float *__restrict__ I)
{
    __shared__ float red[256];
    const int64_t r = blockIdx.x;
    const int n = counts[r];
    for (int w = 0; w < n_win; ++w) {
        const float *src = img + ((size_t)r * n_win + w) * n_dir;
        float m = 0.0f;
        for (int v = threadIdx.x; v < n_dir; v += 256) m = fmaxf(m, src[v]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) I[(size_t)r * n_win + w] = n > 0 ? red[0] / (float)n : 0.0f;
        __syncthreads();
    }
}

// grid (n_win): maximum of I[.][w] over the ROIs
__global__ __launch_bounds__(1024) void k_best(const float *__restrict__ I, int64_t n_roi, int n_win,
                                               float *__restrict__ best)
{
    __shared__ float red[1024];
    const int w = blockIdx.x;
    float m = 0.0f;
    for (int64_t r = threadIdx.x; r < n_roi; r += 1024) m = fmaxf(m, I[(size_t)r * n_win + w]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) best[w] = red[0];
}

__global__ __launch_bounds__(256) void k_keep(const float *__restrict__ I, const float *__restrict__ best,
                                              int64_t n_roi, int n_win, uint32_t mask, float kappa,
                                              int32_t *__restrict__ flag)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n_roi) return;
    int keep = 0;
    for (int w = 0; w < n_win; ++w)
        if (((mask >> w) & 1u) && best[w] > 0.0f && I[(size_t)r * n_win + w] >= kappa * best[w]) keep = 1;
    flag[r] = keep;
}

// one thread per (ROI, sub-cell); kept ROI r writes s^3 rows from pos[r] s^3
__global__ __launch_bounds__(256) void k_emit(const float *__restrict__ centres, const int32_t *__restrict__ flag,
                                              const int64_t *__restrict__ pos, int64_t n_roi, int split,
                                              Offsets off, float *__restrict__ out, int32_t *__restrict__ parent)
{
    const int s3 = split * split * split;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t r = t / s3;
    if (r >= n_roi || !flag[r]) return;
    const int c = (int)(t - r * s3);
    const int i = c / (split * split), j = (c / split) % split, k = c % split;
    const int64_t o = pos[r] * s3 + c;
    out[3 * o] = centres[3 * r] + off.d[i];
    out[3 * o + 1] = centres[3 * r + 1] + off.d[j];
    out[3 * o + 2] = centres[3 * r + 2] + off.d[k];
    if (parent) parent[o] = (int32_t)r;
}

}  // namespace roigrid
}  // namespace ar

extern "C" ar_status ar_refine_roi_grid(ar_context *ctx, const float *centres, const float *images,
                                        const int32_t *counts, int64_t n_roi, int32_t n_win, int32_t n_dir,
                                        uint32_t window_mask, float kappa, float h, int32_t split,
                                        float *out_centres, int32_t *out_parent, int64_t cap, int64_t *n_out,
                                        void *stream)
{
    using namespace ar::roigrid;
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(centres && images && counts && n_out, "centres/images/counts/n_out must not be NULL");
    AR_CHECK(n_roi >= 1 && n_roi < (int64_t)INT32_MAX, "n_roi out of range");
    AR_CHECK(n_win >= 1 && n_win <= kMaxWin, "n_win must be in [1, %d]", kMaxWin);
    AR_CHECK(n_dir >= 1, "n_dir must be >= 1");
    AR_CHECK(split >= 1 && split <= kMaxSplit, "split must be in [1, %d]", kMaxSplit);
    AR_CHECK(h > 0.0f && isfinite(h) && isfinite(kappa), "h must be finite and > 0, kappa finite");
    AR_CHECK(cap == 0 || out_centres != nullptr, "out_centres is NULL");
    *n_out = 0;
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ar::DeviceBuffer I, best, flag, pos, temp;
    AR_TRY(I.reserve(sizeof(float) * n_roi * n_win));
    AR_TRY(best.reserve(sizeof(float) * n_win));
    AR_TRY(flag.reserve(sizeof(int32_t) * n_roi));
    AR_TRY(pos.reserve(sizeof(int64_t) * (n_roi + 1)));
    AR_TRY(temp.reserve(sizeof(int64_t) * ar::scan::tiles(n_roi) + 16));

    k_intensity<<<(unsigned)n_roi, 256, 0, s>>>(images, counts, n_win, n_dir, I.as<float>());
    AR_HIP(hipGetLastError());
    k_best<<<(unsigned)n_win, 1024, 0, s>>>(I.as<float>(), n_roi, n_win, best.as<float>());
    AR_HIP(hipGetLastError());
    k_keep<<<(unsigned)((n_roi + 255) / 256), 256, 0, s>>>(I.as<float>(), best.as<float>(), n_roi, n_win, window_mask,
                                                           kappa, flag.as<int32_t>());
    AR_HIP(hipGetLastError());
    // exclusive scan of the n_roi flags: pos[r] = kept ROIs before r, pos[n_roi] = kept ROIs
    AR_TRY((ar::scan::exclusive_scan<int32_t, int64_t>(flag.as<int32_t>(), n_roi, pos.as<int64_t>(),
                                                       temp.as<int64_t>(), s)));
    int64_t kept = 0;
    AR_HIP(hipMemcpyAsync(&kept, pos.as<int64_t>() + n_roi, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    AR_HIP(hipStreamSynchronize(s));
    const int64_t s3 = (int64_t)split * split * split;
    const int64_t total = kept * s3;
    *n_out = total;
    AR_CHECK(cap >= total, "out capacity %lld is smaller than the %lld refined ROIs", (long long)cap,
             (long long)total);
    if (total == 0) return AR_OK;
    Offsets off;
    for (int i = 0; i < kMaxSplit; ++i)
        off.d[i] = i < split ? (float)((double)h * (double)(2 * i + 1 - split) / (double)(2 * split)) : 0.0f;
    const int64_t threads = n_roi * s3;
    AR_CHECK((threads + 255) / 256 < (int64_t)INT32_MAX, "too many ROIs");
    k_emit<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(centres, flag.as<int32_t>(), pos.as<int64_t>(), n_roi,
                                                             split, off, out_centres, out_parent);
    AR_HIP(hipGetLastError());
    // the local buffers are freed on return; hipFree waits for the kernels
    return AR_OK;
}
