// Real-space signatures (Sec. 2.2, RSP paragraph, Eq. (1); supplement,
// "Controlled windowing of the SDMs", "Sequential implementation tricks",
// reconstruction parameters): per (ROI, direction) an Eq. (1) histogram,
// its Fourier amplitude spectrum and the maximum amplitude in each window.
//
// gfx950 design.  A workgroup of four wavefronts works on one ROI at a time:
// the ROI's relative coordinates are staged once in LDS (larger ROIs in
// chunks), each wavefront takes whole directions (wave-uniform, in SGPRs)
// and reads every atom from the stage with one 16-byte LDS load.  The
// histogram is a wave-private int32 array in LDS filled with LDS integer
// atomics.  The 2^m-point real FFT is one 2^(m-1)-point complex
// Stockham FFT in place in the same LDS (radix-8 passes, twiddle factors per
// lane in registers), and its last stage is evaluated only for the spectrum
// bins the windows cover, fused with the real-input post-processing and
// |X_k|.  Window maxima are a 16-lane DPP reduction.  No workgroup barrier is
// needed for a ROI whose atoms fit the stage.
//
// Two launch forms share that per-direction code:
//   plain       one workgroup per (ROI, direction tile), hardware dispatch;
//   persistent  CU-filling grid whose workgroups pull (ROI, direction chunk)
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

constexpr int kWaves = 4;             // wavefronts per workgroup
constexpr int kStageMult = 256;       // stage capacity granularity (atoms)
constexpr int kStageMax = 4096;

// LDS: the atom stage (cap float4), per wavefront the histogram / FFT buffer
// (NB floats) and 64 scratch floats (discarded atomics of idle lanes, window
// amplitudes), then a 16-byte item slot.
constexpr size_t wave_bytes(int nb) { return (size_t)nb * 4 + 256; }
__host__ __device__ constexpr size_t slot_offset(int nb, int cap) { return (size_t)cap * 16 + (size_t)kWaves * wave_bytes(nb); }
size_t lds_for(int nbins, int cap) { return slot_offset(nbins, cap) + 16; }

// Per-lane constants of the transform, loaded once per kernel.
template <int LOGNB> struct LaneConsts {
    static constexpr int NB = 1 << LOGNB;
    static constexpr int NC = NB / 2;
    static constexpr int R_LAST = FftPlan<NC>::R_LAST;
    PassTwiddles<NB, 8> tw8;
    PassTwiddles<NB, 64> tw64;
    float2 ftw[R_LAST - 1];   // w^(t k), w = exp(-2 pi i / NC), k = this lane's bin
    float2 wk;                // exp(-2 pi i k / NB)
    int mm1, mm2;             // last-stage base indices of k and NC - k
    int mmx;                  // split last stage: this lane's base (mm1 below lane 32, mm2 above)
    int rd;                   // row reduction: scratch slot read by this lane

    __device__ __forceinline__ void load_bin(const float2 *__restrict__ Wg, int kk)
    {
        constexpr int NS = FftPlan<NC>::NS_LAST;
        mm1 = last_base<NS>(kk & (NS - 1));
        mm2 = last_base<NS>((NC - kk) & (NS - 1));
#pragma unroll
        for (int t = 1; t < R_LAST; ++t) ftw[t - 1] = Wg[(2 * t * kk) & (NB - 1)];
        wk = Wg[kk];
    }

    // split last stage (windows within 32 bins): lane l and l + 32 share
    // bin k = kmin + l; the upper lane sums Z_(NC-k) with conjugate twiddles
    __device__ __forceinline__ void load_split(const float2 *__restrict__ Wg, int kk, bool upper)
    {
        load_bin(Wg, kk);
        mmx = upper ? mm2 : mm1;
        if (upper) {
#pragma unroll
            for (int t = 1; t < R_LAST; ++t) ftw[t - 1].y = -ftw[t - 1].y;
        }
    }

    __device__ __forceinline__ void load(const float2 *__restrict__ Wg, const WindowSet &ws, int lane)
    {
        if constexpr (FftPlan<NC>::NS_LAST > 8) tw8.load(Wg, lane);
        if constexpr (FftPlan<NC>::NS_LAST > 64) tw64.load(Wg, lane);
        if (ws.rows == 2) load_split(Wg, min(ws.kmin + (lane & 31), ws.kmax), lane >= 32);
        else load_bin(Wg, min(ws.kmin + lane, ws.kmax));
        // row w = lane / 16 reads window w, bin lo_w + min(lane % 16, width - 1)
        rd = 0;
        const int w = lane >> 4, i = lane & 15;
        for (int u = 0; u < ws.n && u < 4; ++u)
            if (w == u) rd = ws.lo[u] - ws.kmin + min(i, ws.hi[u] - ws.lo[u]);
    }
};

// Stage atoms [first, first + n) of a ROI into LDS (all threads of the
// workgroup; the caller synchronises).  With q = n / 64, the first 64 q
// atoms are stored transposed, atom l q + a at slot a * 64 + l (a < q,
// l < 64), so the 64 lanes binning one slot group take atoms q apart in the
// ROI's order.  That order is cell-sorted: neighbours in it are neighbours
// in space, whose projections crowd into the same histogram bins and banks,
// and the LDS atomics of one instruction then serialise.  The remaining
// n - 64 q atoms (fewer than 64) keep their order at slots 64 q .. n - 1.
// The histogram is a sum of integer counts, the same in any order.
__device__ __forceinline__ void stage_atoms(float4 *xs, const float4 *__restrict__ rel, int64_t first, int n)
{
    const int q = n / kWave;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = q > 0 ? i / q : 0;
        const int slot = i < q * kWave ? (i - l * q) * kWave + l : i;
        xs[slot] = rel[first + i];
    }
}

// Eq. (1) histogram of n staged atoms (slot a * 64 + lane), added into the
// wave's LDS histogram.  Slots go in groups of four: the four bins are formed
// first and the LDS atomics then issued back to back.  Full groups need no
// test; in the last group lanes past the end add into their discard slot
// hist[NB + lane].  The stage holds a multiple of 256 atoms, so the reads of
// the last group stay inside it.
template <int NB>
__device__ __forceinline__ void bin_staged(const float4 *xs, int n, float vx, float vy, float vz, BinConsts bc,
                                           int *hist, int lane)
{
    constexpr float last = (float)(NB - 1);
    const float4 *p = xs + lane;
    int g = 0;
    for (; (g + 4) * kWave <= n; g += 4, p += 4 * kWave) {
        int b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 x = p[i * kWave];
            b[i] = eq1_bin(vx, vy, vz, x.x, x.y, x.z, bc.shift, bc.scale, last);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(&hist[b[i]], 1);
    }
    if (g * kWave < n) {
        int b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 x = p[i * kWave];
            const int bin = eq1_bin(vx, vy, vz, x.x, x.y, x.z, bc.shift, bc.scale, last);
            b[i] = (g + i) * kWave + lane < n ? bin : NB + lane;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(&hist[b[i]], 1);
    }
}

template <int NB> __device__ __forceinline__ void zero_hist(float *A, int lane)
{
#pragma unroll
    for (int i = 0; i < NB / 4 / kWave; ++i) reinterpret_cast<int4 *>(A)[i * kWave + lane] = make_int4(0, 0, 0, 0);
    wave_lds_sync();
}

// Transform the finished histogram of direction v of ROI r and write its
// window maxima (or, DEBUG, the histogram and the whole spectrum).
template <int LOGNB, bool DEBUG>
__device__ __forceinline__ void finish_direction(float *A, LaneConsts<LOGNB> &lc, const WindowSet &ws,
                                                 const float2 *__restrict__ Wg, int lane, int64_t r, int v,
                                                 int n_dir, float *__restrict__ images,
                                                 int32_t *__restrict__ hist_out, float *__restrict__ amp_out)
{
    constexpr int NB = 1 << LOGNB;
    constexpr int NC = NB / 2;
    wave_lds_sync();
    float2 *Z = reinterpret_cast<float2 *>(A);
    float *scratch = A + NB;
    if constexpr (DEBUG) {
        const size_t d = (size_t)r * n_dir + v;
        for (int i = lane; i < NB; i += kWave) hist_out[d * NB + i] = reinterpret_cast<const int32_t *>(A)[i];
        wave_lds_sync();
        fft_head<NB, NC, 1, true>(Z, lc.tw8, lc.tw64, lane);
        stockham_last_full<NB, NC, FftPlan<NC>::R_LAST, FftPlan<NC>::NS_LAST>(Z, Wg, lane);
        wave_lds_sync();
        for (int k = lane; k <= NC; k += kWave) amp_out[d * (NC + 1) + k] = real_amplitude<NC>(Z, Wg, k);
        wave_lds_sync();
        return;
    }
    fft_head<NB, NC, 1, true>(Z, lc.tw8, lc.tw64, lane);
    wave_lds_sync();
    if (ws.rows) {
        scratch[lane] = ws.rows == 2 ? bin_amplitude_split<NC>(Z, lc.mmx, lc.ftw, lc.wk)
                                     : bin_amplitude<NC>(Z, lc.mm1, lc.mm2, lc.ftw, lc.wk);
        wave_lds_sync();
        const float m = row_max16(scratch[lc.rd]);
        const int w = lane >> 4;
        if ((lane & 15) == 0 && w < ws.n) images[((size_t)r * ws.n + w) * n_dir + v] = m;
        wave_lds_sync();
        return;
    }
    // general windows: bins in chunks of 64, per-lane maxima
    int lo = 0, hi = -1;
    for (int w = 0; w < ws.n; ++w)
        if (lane == w) {
            lo = ws.lo[w];
            hi = ws.hi[w];
        }
    float m = 0.0f;
    for (int kc = ws.kmin; kc <= ws.kmax; kc += kWave) {
        if (kc != ws.kmin) lc.load_bin(Wg, min(kc + lane, ws.kmax));
        scratch[lane] = bin_amplitude<NC>(Z, lc.mm1, lc.mm2, lc.ftw, lc.wk);
        wave_lds_sync();
        const int k0 = max(lo, kc), k1 = min(hi, kc + kWave - 1);
        for (int kk = k0; kk <= k1; ++kk) m = fmaxf(m, scratch[kk - kc]);
        wave_lds_sync();
    }
    if (ws.kmax - ws.kmin >= kWave) lc.load_bin(Wg, min(ws.kmin + lane, ws.kmax));
    if (lane < ws.n) images[((size_t)r * ws.n + lane) * n_dir + v] = m;
}

// Directions [v0, v1) of ROI r (atoms [off0, off0 + nw)) by the four
// wavefronts of the workgroup.  If the ROI fits the stage the caller has
// staged it (staged == true) and the wavefronts run independently; otherwise
// every direction round streams the atoms through the stage in chunks, with
// workgroup barriers around each refill (the round count is uniform, so all
// wavefronts meet every barrier).
template <int LOGNB, bool DEBUG>
__device__ __forceinline__ void process_item(const float4 *__restrict__ rel, int64_t off0, int nw, int64_t r,
                                             int v0, int v1, const float *__restrict__ dirs, int n_dir,
                                             BinConsts bc, const WindowSet &ws, LaneConsts<LOGNB> &lc,
                                             const float2 *__restrict__ Wg, float4 *xs, int cap, float *A,
                                             int wave, int lane, float *__restrict__ images,
                                             int32_t *__restrict__ hist_out, float *__restrict__ amp_out)
{
    constexpr int NB = 1 << LOGNB;
    if (nw <= cap) {
        for (int v = v0 + wave; v < v1; v += kWaves) {
            const float vx = dirs[3 * v], vy = dirs[3 * v + 1], vz = dirs[3 * v + 2];
            zero_hist<NB>(A, lane);
            bin_staged<NB>(xs, nw, vx, vy, vz, bc, reinterpret_cast<int *>(A), lane);
            finish_direction<LOGNB, DEBUG>(A, lc, ws, Wg, lane, r, v, n_dir, images, hist_out, amp_out);
        }
        return;
    }
    for (int vr = v0; vr < v1; vr += kWaves) {
        const int v = vr + wave;
        const bool active = v < v1;
        float vx = 0.f, vy = 0.f, vz = 0.f;
        if (active) {
            vx = dirs[3 * v];
            vy = dirs[3 * v + 1];
            vz = dirs[3 * v + 2];
            zero_hist<NB>(A, lane);
        }
        for (int c0 = 0; c0 < nw; c0 += cap) {
            const int n = min(cap, nw - c0);
            __syncthreads();
            stage_atoms(xs, rel, off0 + c0, n);
            __syncthreads();
            if (active) bin_staged<NB>(xs, n, vx, vy, vz, bc, reinterpret_cast<int *>(A), lane);
        }
        if (active) finish_direction<LOGNB, DEBUG>(A, lc, ws, Wg, lane, r, v, n_dir, images, hist_out, amp_out);
    }
}

// ---------------------------------------------------------------- plain form
template <int LOGNB, bool DEBUG>
__global__ __launch_bounds__(256) void k_signatures_plain(
    const float4 *__restrict__ rel, const int64_t *__restrict__ offsets, const float *__restrict__ dirs, int n_dir,
    int dirs_per_block, int n_tiles, const float2 *__restrict__ Wg, BinConsts bc, WindowSet ws, int cap,
    float *__restrict__ images, int32_t *__restrict__ hist_out, float *__restrict__ amp_out)
{
    constexpr int NB = 1 << LOGNB;
    extern __shared__ __align__(16) unsigned char smem[];
    float4 *xs = reinterpret_cast<float4 *>(smem);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *A = reinterpret_cast<float *>(smem + (size_t)cap * 16 + (size_t)wave * wave_bytes(NB));
    LaneConsts<LOGNB> lc;
    lc.load(Wg, ws, lane);

    const int64_t r = (int64_t)blockIdx.x / n_tiles;
    const int tile = (int)((int64_t)blockIdx.x - r * n_tiles);
    const int64_t off0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - off0);
    const int v0 = tile * dirs_per_block;
    const int v1 = min(v0 + dirs_per_block, n_dir);
    if (nw <= cap) {
        stage_atoms(xs, rel, off0, nw);
        __syncthreads();
    }
    process_item<LOGNB, DEBUG>(rel, off0, nw, r, v0, v1, dirs, n_dir, bc, ws, lc, Wg, xs, cap, A, wave, lane,
                               images, hist_out, amp_out);
}

// ---------------------------------------------------------- persistent form
// Item i covers ROI order[i / chunks] and directions
// [(i % chunks) * dpi, +dpi).  Workgroups fetch items from *counter until
// the queue is empty; every workgroup exits after at most n_items + 1
// fetches.  A ROI that fits the stage is staged once per run of items on it.
template <int LOGNB, int MINW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MINW, 8))) void k_signatures_persistent(
    const float4 *__restrict__ rel, const int64_t *__restrict__ offsets, const int32_t *__restrict__ order,
    int64_t n_items, int chunks, int dpi, const float *__restrict__ dirs, int n_dir, const float2 *__restrict__ Wg,
    BinConsts bc, WindowSet ws, int cap, float *__restrict__ images, unsigned long long *__restrict__ counter)
{
    constexpr int NB = 1 << LOGNB;
    extern __shared__ __align__(16) unsigned char smem[];
    // the item slot lies after the stage and the wave buffers: staging may
    // start while other wavefronts still read the slot
    unsigned long long *slot = reinterpret_cast<unsigned long long *>(smem + slot_offset(NB, cap));
    float4 *xs = reinterpret_cast<float4 *>(smem);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *A = reinterpret_cast<float *>(smem + (size_t)cap * 16 + (size_t)wave * wave_bytes(NB));
    LaneConsts<LOGNB> lc;
    lc.load(Wg, ws, lane);

    int64_t cur = -1;
    for (;;) {
        if (threadIdx.x == 0) *slot = atomicAdd(counter, 1ull);
        __syncthreads();
        const unsigned long long it = *slot;
        const int64_t item = (int64_t)(__builtin_amdgcn_readfirstlane((unsigned)it) |
                                       ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(it >> 32)) << 32));
        if ((unsigned long long)item >= (unsigned long long)n_items) break;
        const int64_t r = order[item / chunks];
        const int c = (int)(item % chunks);
        const int64_t off0 = offsets[r];
        const int nw = (int)(offsets[r + 1] - off0);
        if (nw <= cap && r != cur) {
            stage_atoms(xs, rel, off0, nw);
            __syncthreads();
        }
        cur = nw <= cap ? r : -1;
        const int v0 = c * dpi, v1 = min(v0 + dpi, n_dir);
        process_item<LOGNB, false>(rel, off0, nw, r, v0, v1, dirs, n_dir, bc, ws, lc, Wg, xs, cap, A, wave, lane,
                                   images, nullptr, nullptr);
        __syncthreads();
    }
}

__global__ void k_zero_counter(unsigned long long *c) { *c = 0ull; }

// ------------------------------------------------------------ dispatch
using PlainFn = void (*)(const float4 *, const int64_t *, const float *, int, int, int, const float2 *, BinConsts,
                         WindowSet, int, float *, int32_t *, float *);
using PersFn = void (*)(const float4 *, const int64_t *, const int32_t *, int64_t, int, int, const float *, int,
                        const float2 *, BinConsts, WindowSet, int, float *, unsigned long long *);

template <bool DEBUG> PlainFn plain_kernel(int lognb)
{
    switch (lognb) {
    case 8: return k_signatures_plain<8, DEBUG>;
    case 9: return k_signatures_plain<9, DEBUG>;
    case 10: return k_signatures_plain<10, DEBUG>;
    case 11: return k_signatures_plain<11, DEBUG>;
    default: return k_signatures_plain<12, DEBUG>;
    }
}

// occ: 0 = registers as the compiler allocates them, 4 = at most 128 VGPRs
// (four wavefronts per SIMD; may spill).  Only histograms up to 1024 bins
// have the second form.
PersFn pers_kernel(int lognb, int occ)
{
    switch (lognb) {
    case 8: return occ == 4 ? k_signatures_persistent<8, 4> : k_signatures_persistent<8, 1>;
    case 9: return occ == 4 ? k_signatures_persistent<9, 4> : k_signatures_persistent<9, 1>;
    case 10: return occ == 4 ? k_signatures_persistent<10, 4> : k_signatures_persistent<10, 1>;
    case 11: return k_signatures_persistent<11, 1>;
    default: return k_signatures_persistent<12, 1>;
    }
}

// Workgroups above 64 KiB of LDS must be allowed explicitly.
template <typename Fn> ar_status allow_lds(Fn fn, size_t lds)
{
    if (lds > 65536) AR_HIP(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return AR_OK;
}

// Stage capacity for a largest ROI of `big` atoms: the next multiple of 256,
// at most kStageMax (larger ROIs are streamed through the stage).
int stage_for(int64_t big)
{
    const int64_t c = (std::max<int64_t>(big, 1) + kStageMult - 1) / kStageMult * kStageMult;
    return (int)std::min<int64_t>(c, kStageMax);
}

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
                       int32_t *hist, float *amp, int cap, int dirs_per_block, hipStream_t stream)
{
    const float2 *W = nullptr;
    AR_TRY(ctx->twiddle_table(nbins, &W));
    const BinConsts bc = bin_consts(radius, nbins);
    const bool debug = hist != nullptr || amp != nullptr;
    const int n_tiles = (n_dir + dirs_per_block - 1) / dirs_per_block;
    const int64_t blocks = n_roi * (int64_t)n_tiles;
    AR_CHECK(blocks < (int64_t)INT32_MAX, "too many workgroups (%lld)", (long long)blocks);
    AR_CHECK(cap % sig::kStageMult == 0 && cap >= sig::kStageMult && cap <= sig::kStageMax, "bad stage size %d", cap);
    const size_t lds = sig::lds_for(nbins, cap);
    sig::PlainFn fn = debug ? sig::plain_kernel<true>(log2i(nbins)) : sig::plain_kernel<false>(log2i(nbins));
    AR_TRY(sig::allow_lds(fn, lds));
    fn<<<(unsigned)blocks, sig::kWaves * 64, lds, stream>>>((const float4 *)rel, offsets, directions, n_dir,
                                                           dirs_per_block, n_tiles, W, bc, ws, cap, images, hist,
                                                           amp);
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
    int dpi = 32, cap = 1024, blocks_per_cu = 4, min_waves = 1;
    bool tuned = false;
    int64_t big = 0;          // largest ROI of the ordered batch
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
        int dpi, cap, blocks, min_waves;
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
    p->big = n_roi > 0 ? off[ord[0] + 1] - off[ord[0]] : 0;
    if (!p->tuned) p->cap = sig::stage_for(p->big);
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
    const size_t lds = sig::lds_for(p->nbins, p->cap);
    const int blocks = ctx->cu_count * p->blocks_per_cu;
    sig::k_zero_counter<<<1, 1, 0, stream>>>(p->counter.as<unsigned long long>());
    AR_HIP(hipGetLastError());
    sig::PersFn fn = sig::pers_kernel(log2i(p->nbins), p->min_waves);
    AR_TRY(sig::allow_lds(fn, lds));
    fn<<<blocks, sig::kWaves * 64, lds, stream>>>((const float4 *)rel, offsets, p->order.as<int32_t>(), n_items,
                                                 chunks, p->dpi, directions, p->n_dir, W, bc, ws, p->cap, images,
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
                            1024, 256, (hipStream_t)stream);
}

static ar_status gather_into_ctx(ar_context *ctx, const float *positions, const int32_t *types, int64_t n_atoms,
                                 const float *centres, int64_t n_roi, float radius, uint64_t type_mask,
                                 ar::DeviceBuffer &offs, ar::DeviceBuffer &rel, int64_t *total, hipStream_t stream)
{
    AR_TRY(offs.reserve(sizeof(int64_t) * (n_roi + 1)));
    AR_TRY(ar::gather_csr(ctx, positions, types, n_atoms, centres, n_roi, radius, type_mask, offs.as<int64_t>(),
                          nullptr, 0, total, stream));
    AR_TRY(rel.reserve(sizeof(float4) * (*total + 1)));
    AR_TRY(ar::gather_csr(ctx, positions, types, n_atoms, centres, n_roi, radius, type_mask, offs.as<int64_t>(),
                          rel.as<float>(), *total, total, stream));
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
    AR_TRY(gather_into_ctx(ctx, positions, nullptr, n_atoms, centres, n_roi, radius, ~0ull, ctx->g_offsets,
                           ctx->s_rel, &total, s));
    // register chunk sized to the largest ROI (read back once; the gather
    // already synchronised)
    std::vector<int64_t> off(n_roi + 1);
    AR_HIP(hipMemcpyAsync(off.data(), ctx->g_offsets.ptr, sizeof(int64_t) * (n_roi + 1), hipMemcpyDeviceToHost, s));
    AR_HIP(hipStreamSynchronize(s));
    int64_t big = 0;
    for (int64_t r = 0; r < n_roi; ++r) big = std::max(big, off[r + 1] - off[r]);
    const int cap = ar::sig::stage_for(big);
    if (roi_counts) {
        std::vector<int32_t> cnt(n_roi);
        for (int64_t r = 0; r < n_roi; ++r) cnt[r] = (int32_t)(off[r + 1] - off[r]);
        AR_HIP(hipMemcpyAsync(roi_counts, cnt.data(), sizeof(int32_t) * n_roi, hipMemcpyHostToDevice, s));
        AR_HIP(hipStreamSynchronize(s));
    }
    return ar::launch_plain(ctx, ctx->s_rel.as<float>(), ctx->g_offsets.as<int64_t>(), n_roi, radius, directions,
                            n_dir, nbins, ws, images, nullptr, nullptr, cap, 256, s);
}

ar_status araullo_signatures_typed(ar_context *ctx, const float *positions, const int32_t *types, int64_t n_atoms,
                                   const float *centres, int64_t n_roi, float radius, const uint64_t *type_masks,
                                   int32_t n_ch, const float *directions, int32_t n_dir, int32_t nbins,
                                   const int32_t *windows, int32_t n_win, float *images, int32_t *roi_counts,
                                   void *stream)
{
    AR_TRY(ar::check_sig_args(ctx, n_roi, radius, directions, n_dir, nbins));
    AR_CHECK(images != nullptr, "images is NULL");
    AR_CHECK(type_masks != nullptr && n_ch >= 1 && n_ch <= 64, "need 1..64 type masks");
    AR_CHECK(n_atoms == 0 || types != nullptr, "types is NULL");
    ar::WindowSet ws;
    AR_TRY(ar::make_windows(windows, n_win, nbins, &ws));
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const size_t img_row = (size_t)n_win * n_dir;   // floats per ROI and channel
    AR_TRY(ctx->s_typed.reserve(sizeof(float) * img_row * n_roi));
    std::vector<int64_t> off(n_roi + 1);
    std::vector<int32_t> cnt(roi_counts ? (size_t)n_roi * n_ch : 0);
    for (int32_t c = 0; c < n_ch; ++c) {
        int64_t total = 0;
        AR_TRY(gather_into_ctx(ctx, positions, types, n_atoms, centres, n_roi, radius, type_masks[c], ctx->g_offsets,
                               ctx->s_rel, &total, s));
        AR_HIP(hipMemcpyAsync(off.data(), ctx->g_offsets.ptr, sizeof(int64_t) * (n_roi + 1), hipMemcpyDeviceToHost,
                              s));
        AR_HIP(hipStreamSynchronize(s));
        int64_t big = 0;
        for (int64_t r = 0; r < n_roi; ++r) big = std::max(big, off[r + 1] - off[r]);
        if (roi_counts)
            for (int64_t r = 0; r < n_roi; ++r) cnt[(size_t)r * n_ch + c] = (int32_t)(off[r + 1] - off[r]);
        AR_TRY(ar::launch_plain(ctx, ctx->s_rel.as<float>(), ctx->g_offsets.as<int64_t>(), n_roi, radius, directions,
                                n_dir, nbins, ws, ctx->s_typed.as<float>(), nullptr, nullptr, ar::sig::stage_for(big),
                                256, s));
        // channel c of every ROI: rows of img_row floats at a pitch of n_ch rows
        AR_HIP(hipMemcpy2DAsync(images + (size_t)c * img_row, sizeof(float) * img_row * n_ch, ctx->s_typed.ptr,
                                sizeof(float) * img_row, sizeof(float) * img_row, (size_t)n_roi,
                                hipMemcpyDeviceToDevice, s));
    }
    if (roi_counts) {
        AR_HIP(hipMemcpyAsync(roi_counts, cnt.data(), sizeof(int32_t) * cnt.size(), hipMemcpyHostToDevice, s));
        AR_HIP(hipStreamSynchronize(s));
    }
    return AR_OK;
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
    AR_TRY(gather_into_ctx(ctx, positions, nullptr, n_atoms, centres, n_roi, radius, ~0ull, ctx->g_offsets,
                           ctx->s_rel, &total, s));
    ar::WindowSet ws;
    memset(&ws, 0, sizeof(ws));
    return ar::launch_plain(ctx, ctx->s_rel.as<float>(), ctx->g_offsets.as<int64_t>(), n_roi, radius, directions,
                            n_dir, nbins, ws, nullptr, hist, amp, 1024, 64, s);
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
    p->tuned = false;
    AR_TRY(ar::plan_order(p, offsets, n_roi, s));
    hipEvent_t e0, e1;
    AR_HIP(hipEventCreate(&e0));
    AR_HIP(hipEventCreate(&e1));
    float best = INFINITY;
    int bd = p->dpi, bc = p->cap, bb = p->blocks_per_cu, bw = p->min_waves;
    const int dpis[] = {16, 32, 64, 128};
    const int bpcs[] = {2, 3, 4, 6};
    std::vector<int> occs = {1};
    if (p->nbins <= 1024) occs.push_back(4);
    // stage sizes: one that holds the largest ROI, and smaller ones that let
    // more workgroups share a compute unit (larger ROIs are then streamed)
    std::vector<int> caps = {ar::sig::stage_for(p->big)};
    for (int c : {2048, 1024})
        if (c < caps[0]) caps.push_back(c);
    ar_status st = AR_OK;
    for (int occ : occs)
    for (int cap : caps)
        for (int dpi : dpis)
            for (int bpc : bpcs) {
                if (st != AR_OK) break;
                p->min_waves = occ;
                p->cap = cap;
                p->dpi = std::min(dpi, p->n_dir);
                p->blocks_per_cu = bpc;
                st = ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s);  // warm
                if (st == AR_OK && hipEventRecord(e0, s) != hipSuccess) st = ar::fail(AR_EDEVICE, "event record failed");
                if (st == AR_OK) st = ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s);
                if (st == AR_OK && hipEventRecord(e1, s) != hipSuccess) st = ar::fail(AR_EDEVICE, "event record failed");
                if (st == AR_OK && hipEventSynchronize(e1) != hipSuccess) st = ar::fail(AR_EDEVICE, "event sync failed");
                float ms = 0.f;
                if (st == AR_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = ar::fail(AR_EDEVICE, "event time failed");
                if (st == AR_OK && ms < best) {
                    best = ms;
                    bd = p->dpi;
                    bc = cap;
                    bb = bpc;
                    bw = occ;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    AR_TRY(st);
    p->dpi = bd;
    p->cap = bc;
    p->blocks_per_cu = bb;
    p->min_waves = bw;
    p->tuned = true;
    p->have_key = false;
    return ar::plan_launch(p, rel, offsets, n_roi, radius, directions, ws, images, s);
}

ar_status ar_signature_plan_set_config(ar_plan *p, int32_t dirs_per_item, int32_t atoms_per_stage,
                                       int32_t blocks_per_cu, int32_t min_waves)
{
    AR_CHECK(p != nullptr, "plan is NULL");
    AR_CHECK(dirs_per_item >= 1 && dirs_per_item <= p->n_dir, "dirs_per_item must be in [1, n_dir]");
    AR_CHECK(atoms_per_stage >= ar::sig::kStageMult && atoms_per_stage <= ar::sig::kStageMax &&
                 atoms_per_stage % ar::sig::kStageMult == 0,
             "atoms_per_stage must be a multiple of %d in [%d, %d]", ar::sig::kStageMult, ar::sig::kStageMult,
             ar::sig::kStageMax);
    AR_CHECK(blocks_per_cu >= 1 && blocks_per_cu <= 16, "blocks_per_cu must be in [1, 16]");
    AR_CHECK(min_waves == 1 || (min_waves == 4 && p->nbins <= 1024),
             "min_waves must be 1, or 4 for nbins <= 1024");
    p->min_waves = min_waves;
    p->dpi = dirs_per_item;
    p->cap = atoms_per_stage;
    p->blocks_per_cu = blocks_per_cu;
    p->tuned = true;
    p->have_key = false;
    return AR_OK;
}

ar_status ar_signature_plan_config(const ar_plan *p, int32_t *dirs_per_item, int32_t *atoms_per_stage,
                                   int32_t *blocks_per_cu, int32_t *min_waves)
{
    AR_CHECK(p != nullptr, "plan is NULL");
    if (dirs_per_item) *dirs_per_item = p->dpi;
    if (atoms_per_stage) *atoms_per_stage = p->cap;
    if (blocks_per_cu) *blocks_per_cu = p->blocks_per_cu;
    if (min_waves) *min_waves = p->min_waves;
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
    k.cap = p->cap;
    k.min_waves = p->min_waves;
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
