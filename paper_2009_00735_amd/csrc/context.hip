// Context, errors, workspace and the host-side constants of Eq. (1).
#include <math.h>
#include <stdio.h>

#include "ar_internal.h"

namespace ar {

static thread_local char g_error[1024] = "";

ar_status fail(ar_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { g_error[0] = 0; }

DeviceBuffer::~DeviceBuffer()
{
    if (ptr) (void)hipFree(ptr);
}

ar_status DeviceBuffer::reserve(size_t n)
{
    if (n <= bytes && ptr) return AR_OK;
    if (ptr) {
        AR_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
    }
    size_t want = n < 256 ? 256 : n;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return fail(AR_ENOMEM, "hipMalloc(%zu bytes) failed: %s", want, hipGetErrorString(e));
    }
    bytes = want;
    return AR_OK;
}

bool valid_nbins(int32_t nbins)
{
    return nbins >= 256 && nbins <= 4096 && (nbins & (nbins - 1)) == 0;
}

int log2i(int32_t x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Eq. (1): dR = R / (nbins/2 - 1) is the bin width; the nbins bins span
// [-(R + dR), R + dR].  Both constants are evaluated in FP64 and rounded once.
BinConsts bin_consts(float radius, int nbins)
{
    const double R = (double)radius;
    const double dR = R / (double)(nbins / 2 - 1);
    BinConsts c;
    c.shift = (float)(R + dR);
    c.scale = (float)((double)nbins / (2.0 * R + 2.0 * dR));
    return c;
}

ar_status make_windows(const int32_t *windows, int32_t n_win, int32_t nbins, WindowSet *ws)
{
    AR_CHECK(windows != nullptr, "windows is NULL");
    AR_CHECK(n_win >= 1 && n_win <= kMaxWindows, "n_win must be in [1, %d], got %d", kMaxWindows, n_win);
    ws->n = n_win;
    ws->kmin = nbins;
    ws->kmax = 0;
    for (int w = 0; w < n_win; ++w) {
        int lo = windows[2 * w], hi = windows[2 * w + 1];
        AR_CHECK(lo >= 1 && lo <= hi && hi <= nbins / 2,
                 "window %d = [%d, %d] must satisfy 1 <= k_lo <= k_hi <= nbins/2 = %d", w, lo, hi, nbins / 2);
        ws->lo[w] = lo;
        ws->hi[w] = hi;
        if (lo < ws->kmin) ws->kmin = lo;
        if (hi > ws->kmax) ws->kmax = hi;
    }
    for (int w = n_win; w < kMaxWindows; ++w) ws->lo[w] = ws->hi[w] = 0;
    ws->rows = n_win <= 4 && ws->kmax - ws->kmin < 64;
    for (int w = 0; w < n_win; ++w)
        if (ws->hi[w] - ws->lo[w] >= 16) ws->rows = 0;
    if (ws->rows && ws->kmax - ws->kmin < 32) ws->rows = 2;   // two lanes per bin in the last FFT stage
    return AR_OK;
}

}  // namespace ar

ar_status ar_context::twiddle_table(int nbins, const float2 **out)
{
    auto it = twiddles.find(nbins);
    if (it == twiddles.end()) {
        std::vector<float2> h(nbins);
        const double two_pi = 6.283185307179586476925286766559;
        for (int j = 0; j < nbins; ++j) {
            double a = two_pi * (double)j / (double)nbins;
            h[j] = make_float2((float)cos(a), (float)-sin(a));
        }
        auto buf = std::make_unique<ar::DeviceBuffer>();
        AR_TRY(buf->reserve(sizeof(float2) * nbins));
        AR_HIP(hipMemcpy(buf->ptr, h.data(), sizeof(float2) * nbins, hipMemcpyHostToDevice));
        it = twiddles.emplace(nbins, std::move(buf)).first;
    }
    *out = it->second->as<float2>();
    return AR_OK;
}

extern "C" {

const char *ar_last_error(const ar_context *) { return ar::g_error; }

const char *ar_version(void) { return "araullo-gfx950 0.1"; }

ar_status ar_context_create(int device, ar_context **out)
{
    AR_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    int n = 0;
    AR_HIP(hipGetDeviceCount(&n));
    AR_CHECK(device >= 0 && device < n, "device %d out of range [0, %d)", device, n);
    AR_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    AR_HIP(hipGetDeviceProperties(&prop, device));
    AR_TRY(ar::scratch_setup(device));
    auto *c = new (std::nothrow) ar_context();
    if (!c) return ar::fail(AR_ENOMEM, "context allocation failed");
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    c->lds_per_block = (int)prop.sharedMemPerBlock;
    *out = c;
    return AR_OK;
}

ar_status ar_context_destroy(ar_context *ctx)
{
    if (!ctx) return AR_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    delete ctx;
    return AR_OK;
}

ar_status ar_window_bins(double radius, int32_t nbins, double d_min, double d_max, int32_t *k_lo,
                         int32_t *k_hi)
{
    AR_CHECK(k_lo && k_hi, "k_lo/k_hi is NULL");
    AR_CHECK(ar::valid_nbins(nbins), "nbins must be a power of two in [256, 4096], got %d", nbins);
    AR_CHECK(radius > 0.0, "radius must be > 0");
    AR_CHECK(d_min > 0.0 && d_max >= d_min, "need 0 < d_min <= d_max");
    const double dR = radius / (double)(nbins / 2 - 1);
    const double span = 2.0 * radius + 2.0 * dR;
    const double lo = ceil(span / d_max), hi = floor(span / d_min);
    AR_CHECK(lo >= 1.0 && lo <= hi && hi <= (double)(nbins / 2),
             "spacing interval [%g, %g] maps to an empty or out-of-range window [%g, %g]", d_min, d_max, lo, hi);
    *k_lo = (int32_t)lo;
    *k_hi = (int32_t)hi;
    return AR_OK;
}

}  // extern "C"
