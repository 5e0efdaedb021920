// Real-space signatures (Sec. 2.2, RSP paragraph, Eq. (1); supplement,
// "Controlled windowing of the SDMs", "Sequential implementation tricks",
// reconstruction parameters): per (ROI, direction) an Eq. (1) histogram,
// its Fourier amplitude spectrum and the maximum amplitude in each window.
//
// gfx950 design.  Every wavefront works alone on whole directions: the ROI's
// relative coordinates sit in VGPRs (MAXA atoms per lane, more atoms are
// streamed in chunks of 64*MAXA), the direction is wave-uniform (SGPRs), the
// histogram is a wave-private LDS array filled with LDS atomics, the
// 2^m-point real FFT is one 2^(m-1)-point complex Stockham FFT in the same
// LDS (radix-8 passes, ping-pong between the histogram array and a second
// array, twiddles from a per-workgroup LDS table), and only the window bins of
// the one-sided spectrum are formed.  No workgroup barrier is needed after
// the twiddle table is loaded.
//
// Two launch forms share that per-direction code:
//   plain       one workgroup per (ROI, direction tile), hardware dispatch;
//   persistent  CU-filling grid whose wavefronts pull (ROI, direction chunk)
//               items from a device counter, ROIs ordered by decreasing atom
//               count, replayed as a captured HIP graph.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "sig_device.h"

namespace ar {
namespace sig {

struct Tables {
    const float2 *W;     // exp(-2 pi i m / NB), m < NB
};

// per wave: one buffer holding the histogram (NB ints), then in place the
// FFT (NB/2 float2), followed by 64 slots that take the discarded atomics of
// idle lanes and later the window amplitudes of up to 64 bins at a time
template <int LOGNB> constexpr size_t lds_bytes_per_wave() { return (size_t)(1 << LOGNB) * 4 + 256; }
template <int LOGNB> constexpr size_t lds_bytes_table() { return (size_t)(1 << LOGNB) * 8; }

template <int MAXA>
struct AtomRegs {
    float x[MAXA], y[MAXA], z[MAXA];

    __device__ __forceinline__ void load(const float4 *__restrict__ rel, int64_t off0, int first, int nw, int lane)
    {
#pragma unroll
        for (int a = 0; a < MAXA; ++a) {
            const int i = first + a * kWave + lane;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < nw) p = rel[off0 + i];
            x[a] = p.x;
            y[a] = p.y;
            z[a] = p.z;
        }
    }
};

// Eq. (1) histogram of `rem` atoms held in registers (lane-strided), added
// into the wave's LDS histogram.  Slots go in groups of four: one uniform
// branch per group, the four bins formed first and the LDS atomics then issued
// back to back (no VGPR reuse between them, so no wait on each one).  Lanes
// past the last atom add into per-lane discard slots hist[NB + lane] instead
// of branching.
template <int NB, int MAXA>
__device__ __forceinline__ void bin_atoms(const AtomRegs<MAXA> &at, int rem, float vx, float vy, float vz,
                                          BinConsts bc, int *__restrict__ hist, int lane)
{
    static_assert(MAXA % 4 == 0, "register chunk must be a multiple of 4 slots");
#pragma unroll
    for (int g = 0; g < MAXA; g += 4) {
        if (g * kWave < rem) {
            int b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int a = g + i;
                const int bin = eq1_bin(vx, vy, vz, at.x[a], at.y[a], at.z[a], bc.shift, bc.scale, (float)(NB - 1));
                b[i] = a * kWave + lane < rem ? bin : NB + lane;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) atomicAdd(&hist[b[i]], 1);
        }
    }
}

// One direction, from zeroing the histogram to the window maxima / debug dump.
template <int LOGNB, int MAXA, bool DEBUG>
__device__ __forceinline__ void one_direction(AtomRegs<MAXA> &at, bool resident, const float4 *__restrict__ rel,
                                              int64_t off0, int nw, float vx, float vy, float vz, BinConsts bc,
                                              const WindowSet &ws, const float2 *__restrict__ W, int *A, int lane,
                                              float *win_out /* lane w < n_win: result */,
                                              int32_t *__restrict__ hist_out, float *__restrict__ amp_out)
{
    constexpr int NB = 1 << LOGNB;
    constexpr int NC = NB / 2;
    constexpr int CH = MAXA * kWave;
#pragma unroll
    for (int i = lane; i < NB / 4; i += kWave) reinterpret_cast<int4 *>(A)[i] = make_int4(0, 0, 0, 0);
    wave_lds_sync();
    if (resident) {
        bin_atoms<NB, MAXA>(at, nw, vx, vy, vz, bc, A, lane);
    } else {
        for (int c = 0; c < nw; c += CH) {
            at.load(rel, off0, c, nw, lane);
            bin_atoms<NB, MAXA>(at, nw - c, vx, vy, vz, bc, A, lane);
        }
    }
    wave_lds_sync();
    if constexpr (DEBUG) {
        for (int i = lane; i < NB; i += kWave) hist_out[i] = A[i];
        wave_lds_sync();
    }
    float2 *Z = reinterpret_cast<float2 *>(A);
    fft_inplace<NC, 1, true>(Z, W, lane);
    float *amp = reinterpret_cast<float *>(A + NB);     // 64 scratch slots after the buffer
    if constexpr (DEBUG) {
        for (int k = lane; k <= NC; k += kWave) amp_out[k] = real_amplitude<NC>(Z, W, k);
        wave_lds_sync();
    } else {
        int lo = 0, hi = -1;
        for (int w = 0; w < ws.n; ++w)
            if (lane == w) {
                lo = ws.lo[w];
                hi = ws.hi[w];
            }
        float m = 0.0f;
        for (int kc = ws.kmin; kc <= ws.kmax; kc += kWave) {
            const int k = kc + lane;
            if (k <= ws.kmax) amp[lane] = real_amplitude<NC>(Z, W, k);
            wave_lds_sync();
            const int k0 = max(lo, kc), k1 = min(hi, kc + kWave - 1);
            for (int kk = k0; kk <= k1; ++kk) m = fmaxf(m, amp[kk - kc]);
            wave_lds_sync();
        }
        *win_out = m;
    }
}

// ---------------------------------------------------------------- plain form
template <int LOGNB, int MAXA, bool DEBUG>
__global__ __launch_bounds__(256) void k_signatures_plain(
    const float4 *__restrict__ rel, const int64_t *__restrict__ offsets, const float *__restrict__ dirs, int n_dir,
    int dirs_per_block, int n_tiles, const float2 *__restrict__ Wg, BinConsts bc, WindowSet ws,
    float *__restrict__ images, int32_t *__restrict__ hist_out, float *__restrict__ amp_out)
{
    constexpr int NB = 1 << LOGNB;
    extern __shared__ __align__(16) unsigned char smem[];
    float2 *W = reinterpret_cast<float2 *>(smem);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    unsigned char *mine = smem + lds_bytes_table<LOGNB>() + (size_t)wave * lds_bytes_per_wave<LOGNB>();
    int *A = reinterpret_cast<int *>(mine);
    for (int i = threadIdx.x; i < NB; i += blockDim.x) W[i] = Wg[i];
    __syncthreads();

    const int64_t r = (int64_t)blockIdx.x / n_tiles;
    const int tile = (int)((int64_t)blockIdx.x - r * n_tiles);
    const int64_t off0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - off0);
    const int v0 = tile * dirs_per_block;
    const int v1 = min(v0 + dirs_per_block, n_dir);
    AtomRegs<MAXA> at;
    const bool resident = nw <= MAXA * kWave;
    if (resident) at.load(rel, off0, 0, nw, lane);
    for (int v = v0 + wave; v < v1; v += nwaves) {
        const float vx = dirs[3 * v], vy = dirs[3 * v + 1], vz = dirs[3 * v + 2];
        float m;
        const size_t dbg = ((size_t)r * n_dir + v);
        one_direction<LOGNB, MAXA, DEBUG>(at, resident, rel, off0, nw, vx, vy, vz, bc, ws, W, A, lane, &m,
                                          DEBUG ? hist_out + dbg * NB : nullptr,
                                          DEBUG ? amp_out + dbg * (NB / 2 + 1) : nullptr);
        if (!DEBUG && lane < ws.n) images[((size_t)r * ws.n + lane) * n_dir + v] = m;
    }
}

// ---------------------------------------------------------- persistent form
// Item i covers ROI order[i / chunks] and directions
// [(i % chunks) * dpi, +dpi).  Wavefronts fetch items from *counter until the
// queue is empty; every wavefront exits after at most n_items + 1 fetches.
template <int LOGNB, int MAXA>
__global__ __launch_bounds__(256) void k_signatures_persistent(
    const float4 *__restrict__ rel, const int64_t *__restrict__ offsets, const int32_t *__restrict__ order,
    int64_t n_items, int chunks, int dpi, const float *__restrict__ dirs, int n_dir, const float2 *__restrict__ Wg,
    BinConsts bc, WindowSet ws, float *__restrict__ images, unsigned long long *__restrict__ counter)
{
    constexpr int NB = 1 << LOGNB;
    extern __shared__ __align__(16) unsigned char smem[];
    float2 *W = reinterpret_cast<float2 *>(smem);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned char *mine = smem + lds_bytes_table<LOGNB>() + (size_t)wave * lds_bytes_per_wave<LOGNB>();
    int *A = reinterpret_cast<int *>(mine);
    for (int i = threadIdx.x; i < NB; i += blockDim.x) W[i] = Wg[i];
    __syncthreads();

    AtomRegs<MAXA> at;
    int64_t cur = -1;
    bool resident = false;
    int64_t off0 = 0;
    int nw = 0;
    for (;;) {
        unsigned long long item = 0;
        if (lane == 0) item = atomicAdd(counter, 1ull);
        item = __builtin_amdgcn_readfirstlane((unsigned)item) |
               ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(item >> 32)) << 32);
        if ((int64_t)item >= n_items) break;
        const int64_t r = order[(int64_t)item / chunks];
        const int c = (int)((int64_t)item % chunks);
        if (r != cur) {
            cur = r;
            off0 = offsets[r];
            nw = (int)(offsets[r + 1] - off0);
            resident = nw <= MAXA * kWave;
            if (resident) at.load(rel, off0, 0, nw, lane);
        }
        const int v0 = c * dpi, v1 = min(v0 + dpi, n_dir);
        for (int v = v0; v < v1; ++v) {
            const float vx = dirs[3 * v], vy = dirs[3 * v + 1], vz = dirs[3 * v + 2];
            float m;
            one_direction<LOGNB, MAXA, false>(at, resident, rel, off0, nw, vx, vy, vz, bc, ws, W, A, lane, &m,
                                              nullptr, nullptr);
            if (lane < ws.n) images[((size_t)r * ws.n + lane) * n_dir + v] = m;
        }
    }
}

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

// ------------------------------------------------------------ dispatch
using PlainFn = void (*)(const float4 *, const int64_t *, const float *, int, int, int, const float2 *, BinConsts,
                         WindowSet, float *, int32_t *, float *);
using PersFn = void (*)(const float4 *, const int64_t *, const int32_t *, int64_t, int, int, const float *, int,
                        const float2 *, BinConsts, WindowSet, float *, unsigned long long *);

static const int kMaxaOptions[] = {8, 16, 24, 32};

template <int LOGNB, bool DEBUG> PlainFn plain_for_maxa(int maxa)
{
    switch (maxa) {
    case 8: return k_signatures_plain<LOGNB, 8, DEBUG>;
    case 16: return k_signatures_plain<LOGNB, 16, DEBUG>;
    case 24: return k_signatures_plain<LOGNB, 24, DEBUG>;
    default: return k_signatures_plain<LOGNB, 32, DEBUG>;
    }
}

template <bool DEBUG> PlainFn plain_kernel(int lognb, int maxa)
{
    switch (lognb) {
    case 8: return plain_for_maxa<8, DEBUG>(maxa);
    case 9: return plain_for_maxa<9, DEBUG>(maxa);
    case 10: return plain_for_maxa<10, DEBUG>(maxa);
    case 11: return plain_for_maxa<11, DEBUG>(maxa);
    default: return plain_for_maxa<12, DEBUG>(maxa);
    }
}

template <int LOGNB> PersFn pers_for_maxa(int maxa)
{
    switch (maxa) {
    case 8: return k_signatures_persistent<LOGNB, 8>;
    case 16: return k_signatures_persistent<LOGNB, 16>;
    case 24: return k_signatures_persistent<LOGNB, 24>;
    default: return k_signatures_persistent<LOGNB, 32>;
    }
}

PersFn pers_kernel(int lognb, int maxa)
{
    switch (lognb) {
    case 8: return pers_for_maxa<8>(maxa);
    case 9: return pers_for_maxa<9>(maxa);
    case 10: return pers_for_maxa<10>(maxa);
    case 11: return pers_for_maxa<11>(maxa);
    default: return pers_for_maxa<12>(maxa);
    }
}

// Waves per workgroup: keep the workgroup's LDS (twiddle table + per-wave
// buffers) at or below 64 KiB.
int waves_for(int nbins) { return nbins <= 2048 ? 4 : 1; }
size_t lds_for(int nbins, int waves) { return (size_t)nbins * 8 + (size_t)waves * ((size_t)nbins * 4 + 256); }

}  // namespace sig

ar_status check_sig_args(ar_context *ctx, int64_t n_roi, float radius, const float *directions, int32_t n_dir,
                         int32_t nbins)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(n_roi >= 1, "n_roi must be >= 1");
    AR_CHECK(radius > 0.f && isfinite(radius), "radius must be finite and > 0");
    AR_CHECK(directions != nullptr, "directions is NULL");
    AR_CHECK(n_dir >= 1, "n_dir must be >= 1");
    AR_CHECK(valid_nbins(nbins), "nbins must be a power of two in [256, 4096], got %d", nbins);
    return AR_OK;
}

ar_status launch_plain(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi, float radius,
                       const float *directions, int32_t n_dir, int32_t nbins, const WindowSet &ws, float *images,
                       int32_t *hist, float *amp, int maxa, int dirs_per_block, hipStream_t stream)
{
    const float2 *W = nullptr;
    AR_TRY(ctx->twiddle_table(nbins, &W));
    const BinConsts bc = bin_consts(radius, nbins);
    const bool debug = hist != nullptr || amp != nullptr;
    const int waves = sig::waves_for(nbins);
    const int n_tiles = (n_dir + dirs_per_block - 1) / dirs_per_block;
    const int64_t blocks = n_roi * (int64_t)n_tiles;
    AR_CHECK(blocks < (int64_t)INT32_MAX, "too many workgroups (%lld)", (long long)blocks);
    const size_t lds = sig::lds_for(nbins, waves);
    sig::PlainFn fn = debug ? sig::plain_kernel<true>(log2i(nbins), maxa) : sig::plain_kernel<false>(log2i(nbins), maxa);
    fn<<<(unsigned)blocks, waves * 64, lds, stream>>>((const float4 *)rel, offsets, directions, n_dir, dirs_per_block,
                                                     n_tiles, W, bc, ws, images, hist, amp);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // namespace ar

// ================================================================== plans
struct ar_plan {
    ar_context *ctx = nullptr;
    int64_t max_roi = 0, max_total = 0;
    int32_t n_dir = 0, nbins = 0, n_win = 0;
    // tuned configuration
    int dpi = 32, maxa = 16, waves = 4, blocks_per_cu = 4;
    bool tuned = false;
    // queue
    ar::DeviceBuffer order, counter;
    const int64_t *order_for = nullptr;
    int64_t order_n = -1;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        const void *rel, *offsets, *dirs, *images;
        int64_t n_roi;
        float radius;
        int dpi, maxa, waves, blocks;
        ar::WindowSet ws;
    } key;
    bool have_key = false;
    ~ar_plan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace ar {

static ar_status plan_order(ar_plan *p, const int64_t *offsets, int64_t n_roi, hipStream_t stream)
{
    if (p->order_for == offsets && p->order_n == n_roi) return AR_OK;
    std::vector<int64_t> off(n_roi + 1);
    AR_HIP(hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * (n_roi + 1), hipMemcpyDeviceToHost, stream));
    AR_HIP(hipStreamSynchronize(stream));
    AR_CHECK(off[0] >= 0 && off[n_roi] <= p->max_total, "gathered rows exceed the plan capacity");
    std::vector<int32_t> ord(n_roi);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return off[a + 1] - off[a] > off[b + 1] - off[b];
    });
    AR_TRY(p->order.reserve(sizeof(int32_t) * n_roi));
    AR_HIP(hipMemcpyAsync(p->order.ptr, ord.data(), sizeof(int32_t) * n_roi, hipMemcpyHostToDevice, stream));
    AR_HIP(hipStreamSynchronize(stream));
    p->order_for = offsets;
    p->order_n = n_roi;
    return AR_OK;
}

static ar_status plan_launch(ar_plan *p, const float *rel, const int64_t *offsets, int64_t n_roi, float radius,
                             const float *directions, const WindowSet &ws, float *images, hipStream_t stream)
{
    ar_context *ctx = p->ctx;
    const float2 *W = nullptr;
    AR_TRY(ctx->twiddle_table(p->nbins, &W));
    const BinConsts bc = bin_consts(radius, p->nbins);
    const int chunks = (p->n_dir + p->dpi - 1) / p->dpi;
    const int64_t n_items = n_roi * (int64_t)chunks;
    const size_t lds = sig::lds_for(p->nbins, p->waves);
    const int blocks = ctx->cu_count * p->blocks_per_cu;
    sig::k_zero_counter<<<1, 1, 0, stream>>>(p->counter.as<unsigned long long>());
    AR_HIP(hipGetLastError());
    sig::PersFn fn = sig::pers_kernel(log2i(p->nbins), p->maxa);
    fn<<<blocks, p->waves * 64, lds, stream>>>((const float4 *)rel, offsets, p->order.as<int32_t>(), n_items, chunks,
                                              p->dpi, directions, p->n_dir, W, bc, ws, images,
                                              p->counter.as<unsigned long long>());
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // namespace ar

extern "C" {

ar_status araullo_signatures_csr(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                                 float radius, const float *directions, int32_t n_dir, int32_t nbins,
                                 const int32_t *windows, int32_t n_win, float *images, void *stream)
{
    AR_TRY(ar::check_sig_args(ctx, n_roi, radius, directions, n_dir, nbins));
    AR_CHECK(rel && offsets && images, "rel/offsets/images must not be NULL");
    ar::WindowSet ws;
    AR_TRY(ar::make_windows(windows, n_win, nbins, &ws));
    AR_HIP(hipSetDevice(ctx->device));
    return ar::launch_plain(ctx, rel, offsets, n_roi, radius, directions, n_dir, nbins, ws, images, nullptr, nullptr,
                            16, 256, (hipStream_t)stream);
}

static ar_status gather_into_ctx(ar_context *ctx, const float *positions, int64_t n_atoms, const float *centres,
                                 int64_t n_roi, float radius, ar::DeviceBuffer &offs, ar::DeviceBuffer &rel,
                                 int64_t *total, hipStream_t stream)
{
    AR_TRY(offs.reserve(sizeof(int64_t) * (n_roi + 1)));
    AR_TRY(ar::gather_csr(ctx, positions, n_atoms, centres, n_roi, radius, offs.as<int64_t>(), nullptr, 0, total,
                          stream));
    AR_TRY(rel.reserve(sizeof(float4) * (*total + 1)));
    AR_TRY(ar::gather_csr(ctx, positions, n_atoms, centres, n_roi, radius, offs.as<int64_t>(), rel.as<float>(),
                          *total, total, stream));
    return AR_OK;
}

ar_status araullo_signatures(ar_context *ctx, const float *positions, int64_t n_atoms, const float *centres,
                             int64_t n_roi, float radius, const float *directions, int32_t n_dir, int32_t nbins,
                             const int32_t *windows, int32_t n_win, float *images, int32_t *roi_counts, void *stream)
{
    AR_TRY(ar::check_sig_args(ctx, n_roi, radius, directions, n_dir, nbins));
    AR_CHECK(images != nullptr, "images is NULL");
    ar::WindowSet ws;
    AR_TRY(ar::make_windows(windows, n_win, nbins, &ws));
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    AR_TRY(gather_into_ctx(ctx, positions, n_atoms, centres, n_roi, radius, ctx->g_offsets, ctx->s_rel, &total, s));
    // register chunk sized to the largest ROI (read back once; the gather
    // already synchronised)
    std::vector<int64_t> off(n_roi + 1);
    AR_HIP(hipMemcpyAsync(off.data(), ctx->g_offsets.ptr, sizeof(int64_t) * (n_roi + 1), hipMemcpyDeviceToHost, s));
    AR_HIP(hipStreamSynchronize(s));
    int64_t big = 0;
    for (int64_t r = 0; r < n_roi; ++r) big = std::max(big, off[r + 1] - off[r]);
    int maxa = 32;
    for (int m : ar::sig::kMaxaOptions)
        if ((int64_t)m * 64 >= big) {
            maxa = m;
            break;
        }
    if (roi_counts) {
        std::vector<int32_t> cnt(n_roi);
        for (int64_t r = 0; r < n_roi; ++r) cnt[r] = (int32_t)(off[r + 1] - off[r]);
        AR_HIP(hipMemcpyAsync(roi_counts, cnt.data(), sizeof(int32_t) * n_roi, hipMemcpyHostToDevice, s));
        AR_HIP(hipStreamSynchronize(s));
    }
    return ar::launch_plain(ctx, ctx->s_rel.as<float>(), ctx->g_offsets.as<int64_t>(), n_roi, radius, directions,
                            n_dir, nbins, ws, images, nullptr, nullptr, maxa, 256, s);
}

ar_status araullo_sdm(ar_context *ctx, const float *positions, int64_t n_atoms, const float *centres, int64_t n_roi,
                      float radius, const float *directions, int32_t n_dir, int32_t nbins, int32_t *hist, float *amp,
                      void *stream)
{
    AR_TRY(ar::check_sig_args(ctx, n_roi, radius, directions, n_dir, nbins));
    AR_CHECK(hist != nullptr && amp != nullptr, "hist and amp must both be given");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    AR_TRY(gather_into_ctx(ctx, positions, n_atoms, centres, n_roi, radius, ctx->g_offsets, ctx->s_rel, &total, s));
    ar::WindowSet ws;
    memset(&ws, 0, sizeof(ws));
    return ar::launch_plain(ctx, ctx->s_rel.as<float>(), ctx->g_offsets.as<int64_t>(), n_roi, radius, directions,
                            n_dir, nbins, ws, nullptr, hist, amp, 8, 64, s);
}

ar_status ar_signature_plan_create(ar_context *ctx, int64_t max_roi, int64_t max_total, int32_t n_dir, int32_t nbins,
                                   int32_t n_win, ar_plan **out)
{
    AR_CHECK(ctx && out, "ctx/out is NULL");
    *out = nullptr;
    AR_CHECK(max_roi >= 1 && max_total >= 0, "bad capacity");
    AR_CHECK(n_dir >= 1, "n_dir must be >= 1");
    AR_CHECK(ar::valid_nbins(nbins), "nbins must be a power of two in [256, 4096]");
    AR_CHECK(n_win >= 1 && n_win <= ar::kMaxWindows, "n_win out of range");
    AR_HIP(hipSetDevice(ctx->device));
    auto *p = new (std::nothrow) ar_plan();
    if (!p) return ar::fail(AR_ENOMEM, "plan allocation failed");
    p->ctx = ctx;
    p->max_roi = max_roi;
    p->max_total = max_total;
    p->n_dir = n_dir;
    p->nbins = nbins;
    p->n_win = n_win;
    p->waves = ar::sig::waves_for(nbins);
    ar_status s = p->order.reserve(sizeof(int32_t) * max_roi);
    if (s == AR_OK) s = p->counter.reserve(sizeof(unsigned long long));
    if (s != AR_OK) {
        delete p;
        return s;
    }
    *out = p;
    return AR_OK;
}

ar_status ar_signature_plan_destroy(ar_plan *plan)
{
    if (!plan) return AR_OK;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipDeviceSynchronize();
    delete plan;
    return AR_OK;
}

static ar_status plan_check(ar_plan *p, const float *rel, const int64_t *offsets, int64_t n_roi, float radius,
                            const float *directions, const int32_t *windows, float *images, ar::WindowSet *ws)
{
    AR_CHECK(p != nullptr, "plan is NULL");
    AR_CHECK(rel && offsets && directions && images, "rel/offsets/directions/images must not be NULL");
    AR_CHECK(n_roi >= 1 && n_roi <= p->max_roi, "n_roi must be in [1, %lld]", (long long)p->max_roi);
    AR_CHECK(radius > 0.f && isfinite(radius), "radius must be finite and > 0");
    AR_TRY(ar::make_windows(windows, p->n_win, p->nbins, ws));
    return AR_OK;
}

ar_status ar_signature_plan_tune(ar_plan *p, const float *rel, const int64_t *offsets, int64_t n_roi, float radius,
                                 const float *directions, const int32_t *windows, float *images, void *stream)
{
    ar::WindowSet ws;
    AR_TRY(plan_check(p, rel, offsets, n_roi, radius, directions, windows, images, &ws));
    AR_HIP(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    AR_TRY(ar::plan_order(p, offsets, n_roi, s));
    hipEvent_t e0, e1;
    AR_HIP(hipEventCreate(&e0));
    AR_HIP(hipEventCreate(&e1));
    float best = INFINITY;
    int bd = p->dpi, bm = p->maxa, bb = p->blocks_per_cu;
    const int dpis[] = {8, 16, 32, 64};
    const int bpcs[] = {2, 4, 8};
    // register chunks below the largest ROI would stream atoms: only try
    // chunks that hold it, plus the next smaller one
    std::vector<int64_t> off(n_roi + 1);
    AR_HIP(hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * (n_roi + 1), hipMemcpyDeviceToHost, s));
    AR_HIP(hipStreamSynchronize(s));
    int64_t big = 0;
    for (int64_t r = 0; r < n_roi; ++r) big = std::max(big, off[r + 1] - off[r]);
    for (int maxa : ar::sig::kMaxaOptions)
        for (int dpi : dpis)
            for (int bpc : bpcs) {
                if ((int64_t)maxa * 64 * 2 < big) continue;
                p->maxa = maxa;
                p->dpi = dpi;
                p->blocks_per_cu = bpc;
                AR_TRY(ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s));  // warm
                AR_HIP(hipEventRecord(e0, s));
                AR_TRY(ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s));
                AR_HIP(hipEventRecord(e1, s));
                AR_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                AR_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    bd = dpi;
                    bm = maxa;
                    bb = bpc;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->dpi = bd;
    p->maxa = bm;
    p->blocks_per_cu = bb;
    p->tuned = true;
    p->have_key = false;
    return ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s);
}

ar_status ar_signature_plan_set_config(ar_plan *p, int32_t dirs_per_item, int32_t atoms_per_lane,
                                       int32_t blocks_per_cu)
{
    AR_CHECK(p != nullptr, "plan is NULL");
    AR_CHECK(dirs_per_item >= 1 && dirs_per_item <= p->n_dir, "dirs_per_item must be in [1, n_dir]");
    AR_CHECK(atoms_per_lane == 8 || atoms_per_lane == 16 || atoms_per_lane == 24 || atoms_per_lane == 32,
             "atoms_per_lane must be 8, 16, 24 or 32");
    AR_CHECK(blocks_per_cu >= 1 && blocks_per_cu <= 16, "blocks_per_cu must be in [1, 16]");
    p->dpi = dirs_per_item;
    p->maxa = atoms_per_lane;
    p->blocks_per_cu = blocks_per_cu;
    p->tuned = true;
    p->have_key = false;
    return AR_OK;
}

ar_status ar_signature_plan_config(const ar_plan *p, int32_t *dirs_per_item, int32_t *atoms_per_lane,
                                   int32_t *waves_per_group)
{
    AR_CHECK(p != nullptr, "plan is NULL");
    if (dirs_per_item) *dirs_per_item = p->dpi;
    if (atoms_per_lane) *atoms_per_lane = p->maxa;
    if (waves_per_group) *waves_per_group = p->waves;
    return AR_OK;
}

ar_status ar_signature_plan_run(ar_plan *p, const float *rel, const int64_t *offsets, int64_t n_roi, float radius,
                                const float *directions, const int32_t *windows, float *images, int32_t use_graph,
                                void *stream)
{
    ar::WindowSet ws;
    AR_TRY(plan_check(p, rel, offsets, n_roi, radius, directions, windows, images, &ws));
    AR_HIP(hipSetDevice(p->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    AR_TRY(ar::plan_order(p, offsets, n_roi, s));
    if (!use_graph) return ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s);
    ar_plan::Key k;
    memset(&k, 0, sizeof(k));
    k.rel = rel;
    k.offsets = offsets;
    k.dirs = directions;
    k.images = images;
    k.n_roi = n_roi;
    k.radius = radius;
    k.dpi = p->dpi;
    k.maxa = p->maxa;
    k.waves = p->waves;
    k.blocks = p->blocks_per_cu;
    k.ws = ws;
    if (!p->have_key || memcmp(&k, &p->key, sizeof(k)) != 0) {
        if (p->exec) {
            AR_HIP(hipGraphExecDestroy(p->exec));
            p->exec = nullptr;
        }
        if (p->graph) {
            AR_HIP(hipGraphDestroy(p->graph));
            p->graph = nullptr;
        }
        // capture on a private stream so the caller's stream may be the null stream
        hipStream_t cs;
        AR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        AR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        ar_status st = ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (st != AR_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        AR_HIP(e);
        p->graph = g;
        AR_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        p->key = k;
        p->have_key = true;
    }
    AR_HIP(hipGraphLaunch(p->exec, s));
    return AR_OK;
}

}  // extern "C"
