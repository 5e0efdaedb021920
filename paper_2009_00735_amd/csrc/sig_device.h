// Device building blocks of the real-space signature kernels (Sec. 2.2,
// Eq. (1); supplement "Controlled windowing of the SDMs" and "Sequential
// implementation tricks": FFT of each histogram in single precision using
// conjugate-even symmetry).  Included by signatures.hip only.
//
// This translation unit is compiled with -ffp-contract=off: the Eq. (1)
// projection must round exactly as mul, fma, fma, add, mul; every fused
// multiply-add in the FFT is written out with fmaf.
#pragma once

#include "ar_internal.h"

namespace ar {
namespace sig {

constexpr int kWave = 64;

__device__ __forceinline__ void wave_lds_sync()
{
    // LDS operations of one wavefront complete in issue order; this keeps the
    // compiler from moving LDS accesses across the point.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// acc + a * b and acc + a * conj(b)
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b)
{
    return make_float2(fmaf(-a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(a.y, b.x, fmaf(a.x, b.y, acc.y)));
}
__device__ __forceinline__ float2 cmac_conj(float2 acc, float2 a, float2 b)
{
    return make_float2(fmaf(a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(-a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// In-register forward DFTs (exp(-2 pi i s t / R)).
__device__ __forceinline__ void dft2(float2 *v)
{
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const float2 s13 = cadd(a1, a3), d13 = cmul_mi(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

__device__ __forceinline__ void dft4(float2 *v) { dft4(v[0], v[1], v[2], v[3]); }

__device__ __forceinline__ void dft8(float2 *v)
{
    const float h = 0.70710678118654752440f;
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    // o_t *= exp(-2 pi i t / 8)
    o1 = make_float2((o1.x + o1.y) * h, (o1.y - o1.x) * h);
    o2 = cmul_mi(o2);
    o3 = make_float2((o3.y - o3.x) * h, -(o3.x + o3.y) * h);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int R> __device__ __forceinline__ void dftR(float2 *v)
{
    if constexpr (R == 8) dft8(v);
    else if constexpr (R == 4) dft4(v);
    else dft2(v);
}

// Swizzled float2 layout of the FFT buffer: element i lives at
// i ^ h(i >> 5), h(x) = (x & 7) | (((x >> 1) & 3) << 3).  Within each aligned
// block of 32 elements this is a bijection.  Reads of a pass touch 32
// consecutive elements per half-wavefront (XOR by a constant: still one
// element per bank pair); the strided writes of the first two passes land on
// 32 distinct bank pairs (low bits taken by the stride XORed with the block
// index), so no pass has LDS bank conflicts.
__device__ __forceinline__ int swz(int i)
{
    const int x = i >> 5;
    return i ^ ((x & 7) | (((x >> 1) & 3) << 3));
}

// Radix plan of the NC-point complex transform: radix-8 passes on
// sub-transform lengths NS = 1, 8, 64, ... while more than a factor 8 is
// left, then one last stage of radix NC / NS_LAST (2, 4 or 8).  Every pass
// before the last has NS <= 64, so the twiddle factor of butterfly j,
// exp(-2 pi i t (j mod NS) / (8 NS)), depends on the lane only
// (j mod NS = lane mod NS): each lane keeps those factors in registers.
template <int NC> struct FftPlan {
    static constexpr int last_ns()
    {
        int ns = 1;
        while (NC / ns > 8) ns *= 8;
        return ns;
    }
    static constexpr int NS_LAST = last_ns();
    static constexpr int R_LAST = NC / NS_LAST;
    static_assert(NS_LAST <= 512, "transform length out of range");
};

// Per-lane twiddle factors of one radix-8 pass with sub-transform length NS
// (NS = 8 or 64), taken from the NB-point table Wg[m] = exp(-2 pi i m / NB).
template <int NB, int NS> struct PassTwiddles {
    float2 w[7];
    __device__ __forceinline__ void load(const float2 *__restrict__ Wg, int lane)
    {
        constexpr int STRIDE = NB / (NS * 8);
        const int k = lane & (NS - 1);
#pragma unroll
        for (int t = 1; t < 8; ++t) w[t - 1] = Wg[(t * k * STRIDE) & (NB - 1)];
    }
};

// One in-place Stockham autosort pass of radix R on NC complex points in
// LDS, sub-transform length NS before the pass.  Butterfly j reads element
// j + t NC/R, applies twiddles exp(-2 pi i t (j mod NS)/(NS R)) (tw[t-1],
// the same for every butterfly of a lane) and writes element
// (j - j mod NS) R + j mod NS + t NS.  Every lane loads the inputs of all its
// butterflies before any write; LDS operations of a wavefront execute in
// order, so the pass can overwrite its own input.  FROM_HIST: the input is
// the int32 histogram read unswizzled as pairs (h_2n, h_2n+1) = z_n.
template <int NC, int R, int NS, bool FROM_HIST>
__device__ __forceinline__ void stockham_pass(float2 *buf, const float2 *tw, int lane)
{
    constexpr int NBF = NC / R;
    constexpr int PER = (NBF + kWave - 1) / kWave;   // butterflies per lane
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = p * kWave + lane;
        if (NBF % kWave == 0 || j < NBF) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if constexpr (FROM_HIST) {
                    const int2 q = reinterpret_cast<const int2 *>(buf)[j + t * NBF];
                    v[p][t] = make_float2((float)q.x, (float)q.y);
                } else {
                    v[p][t] = buf[swz(j + t * NBF)];
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = p * kWave + lane;
        if (NBF % kWave == 0 || j < NBF) {
            const int k = j & (NS - 1);
            if constexpr (NS > 1) {
#pragma unroll
                for (int t = 1; t < R; ++t) v[p][t] = cmul(v[p][t], tw[t - 1]);
            }
            dftR<R>(v[p]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[swz(base + t * NS)] = v[p][t];
        }
    }
}

// The last stage in full (every output), twiddles read from the global
// table; used only where the whole spectrum is written out.
template <int NB, int NC, int R, int NS>
__device__ __forceinline__ void stockham_last_full(float2 *buf, const float2 *__restrict__ Wg, int lane)
{
    constexpr int NBF = NC / R;
    constexpr int PER = (NBF + kWave - 1) / kWave;
    constexpr int STRIDE = NB / (NS * R);
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = p * kWave + lane;
        if (NBF % kWave == 0 || j < NBF) {
#pragma unroll
            for (int t = 0; t < R; ++t) v[p][t] = buf[swz(j + t * NBF)];
        }
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = p * kWave + lane;
        if (NBF % kWave == 0 || j < NBF) {
            const int k = j & (NS - 1);
#pragma unroll
            for (int t = 1; t < R; ++t) v[p][t] = cmul(v[p][t], Wg[(t * k * STRIDE) & (NB - 1)]);
            dftR<R>(v[p]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[swz(base + t * NS)] = v[p][t];
        }
    }
}

// All passes before the last stage.
template <int NB, int NC, int NS, bool FROM_HIST>
__device__ __forceinline__ void fft_head(float2 *buf, const PassTwiddles<NB, 8> &tw8,
                                         const PassTwiddles<NB, 64> &tw64, int lane)
{
    if constexpr (NS < FftPlan<NC>::NS_LAST) {
        const float2 *tw = NS == 8 ? tw8.w : tw64.w;
        stockham_pass<NC, 8, NS, FROM_HIST>(buf, tw, lane);
        wave_lds_sync();
        fft_head<NB, NC, NS * 8, false>(buf, tw8, tw64, lane);
    }
}

// Element index of Y_t[m] (element t NS + m) in the swizzled layout.  For
// NS = 64: t NS + m has block index 2t + (m >> 5), so the swizzle XORs m with
// (m >> 5) ^ 10 (t mod 4): one XOR per t mod 4 and the rest an immediate
// offset (mm = m ^ (m >> 5) is per lane).  For NS >= 256 the block index of
// t NS + m agrees with that of m in the swizzled bits, so the element is
// swz(m) + t NS.
template <int NS> __device__ __forceinline__ int last_index(int mm, int t)
{
    if constexpr (NS == 64) return (mm ^ (10 * (t & 3))) + 64 * t;
    else if constexpr (NS >= 256) return mm + NS * t;
    else return swz(t * NS + mm);
}
template <int NS> __device__ __forceinline__ int last_base(int m)
{
    if constexpr (NS == 64) return m ^ (m >> 5);
    else if constexpr (NS >= 256) return swz(m);
    else return m;
}

// Last stage restricted to the outputs one real-spectrum bin needs.  After
// the earlier passes the buffer holds R sub-transforms Y_t of length NS
// (element t NS + m), and the packed transform is
//   Z_k = sum_t Y_t[k mod NS] w^(t k),  w = exp(-2 pi i / NC),
// so Z_k and Z_(NC-k) (twiddles conj(w^(t k))) come from 2R reads and
// R - 1 complex multiply-adds each.  Then, with E = (Z_k + conj Z_(NC-k))/2
// and O = -i (Z_k - conj Z_(NC-k))/2, X_k = E + exp(-2 pi i k / NB) O and the
// result is |X_k|.  mm1, mm2: last_base of k mod NS and (NC - k) mod NS;
// ftw[t-1] = w^(t k), wk = exp(-2 pi i k / NB).
template <int NC>
__device__ __forceinline__ float bin_amplitude(const float2 *buf, int mm1, int mm2, const float2 *ftw, float2 wk)
{
    constexpr int NS = FftPlan<NC>::NS_LAST;
    constexpr int R = FftPlan<NC>::R_LAST;
    float2 a = buf[last_index<NS>(mm1, 0)];
    float2 b = buf[last_index<NS>(mm2, 0)];
#pragma unroll
    for (int t = 1; t < R; ++t) {
        a = cmac(a, buf[last_index<NS>(mm1, t)], ftw[t - 1]);
        b = cmac_conj(b, buf[last_index<NS>(mm2, t)], ftw[t - 1]);
    }
    // 2E = Z_k + conj Z', 2O = -i (Z_k - conj Z')
    const float2 e2 = make_float2(a.x + b.x, a.y - b.y);
    const float2 o2 = make_float2(a.y + b.y, b.x - a.x);
    const float2 x2 = cmac(e2, o2, wk);
    return 0.5f * sqrtf(fmaf(x2.x, x2.x, x2.y * x2.y));
}

// The same |X_k| with the two R-term sums on two lanes: lane l < 32 sums
// Z_k, lane l + 32 sums Z_(NC-k) (its twiddles conjugated, base mmx = that
// lane's last_base), and the partial results are exchanged across the
// half-wavefronts.  Valid in lanes 0..31, for windows spanning at most 32
// bins: half the multiply-adds and LDS reads of bin_amplitude.
template <int NC>
__device__ __forceinline__ float bin_amplitude_split(const float2 *buf, int mmx, const float2 *ftw, float2 wk)
{
    constexpr int NS = FftPlan<NC>::NS_LAST;
    constexpr int R = FftPlan<NC>::R_LAST;
    float2 a = buf[last_index<NS>(mmx, 0)];
#pragma unroll
    for (int t = 1; t < R; ++t) a = cmac(a, buf[last_index<NS>(mmx, t)], ftw[t - 1]);
    const float2 b = make_float2(__shfl_xor(a.x, 32), __shfl_xor(a.y, 32));
    const float2 e2 = make_float2(a.x + b.x, a.y - b.y);
    const float2 o2 = make_float2(a.y + b.y, b.x - a.x);
    const float2 x2 = cmac(e2, o2, wk);
    return 0.5f * sqrtf(fmaf(x2.x, x2.x, x2.y * x2.y));
}

// |X_k| of the real input from the full packed transform Z (length NC,
// swizzled): X_k = E_k + exp(-2 pi i k / NB) O_k, 0 <= k <= NC.
template <int NC>
__device__ __forceinline__ float real_amplitude(const float2 *__restrict__ Z, const float2 *__restrict__ Wg, int k)
{
    const float2 zk = Z[swz(k & (NC - 1))];
    const float2 zm = Z[swz((NC - k) & (NC - 1))];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    const float2 x = cadd(e, cmul(Wg[k], o));
    return sqrtf(fmaf(x.x, x.x, x.y * x.y));
}

// Maximum over the 16 lanes of each row of the wavefront (every lane of the
// row receives it): xor-1 and xor-2 quad permutations, then the half-row and
// row mirrors.
__device__ __forceinline__ float row_max16(float x)
{
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false)));
    return x;
}

// Eq. (1) for one atom: bin index, FP32, fixed operation order.  The clamp
// is applied before the conversion: trunc(clamp(t, 0, last)) equals
// clamp(floor(t), 0, last) for every finite t (on [0, last] trunc = floor;
// below 0 both give 0; above last both give last), and the conversion input
// is always in range.
__device__ __forceinline__ int eq1_bin(float vx, float vy, float vz, float dx, float dy, float dz, float shift,
                                       float scale, float last)
{
    const float s = fmaf(vz, dz, fmaf(vy, dy, vx * dx));
    const float t = (s + shift) * scale;
    return (int)__builtin_amdgcn_fmed3f(t, 0.0f, last);
}

}  // namespace sig
}  // namespace ar
