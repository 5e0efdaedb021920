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

// One in-place Stockham autosort pass of radix R on NC complex points in
// LDS, sub-transform length NS before the pass.  Butterfly j reads
// element j + t NC/R, applies twiddles exp(-2 pi i t (j mod NS)/(NS R)) and
// writes element (j - j mod NS) R + j mod NS + t NS.  Every lane loads the
// inputs of all its butterflies before any write; LDS operations of a
// wavefront execute in order, so the pass can overwrite its own input.  The
// twiddle table W holds exp(-2 pi i m / NB), m < NB, NB = 2 NC.  FROM_INT:
// the input is the integer histogram, read unswizzled as pairs
// (h_2n, h_2n+1) = z_n.
template <int NC, int R, int NS, bool FROM_INT>
__device__ __forceinline__ void stockham_pass(float2 *buf, const float2 *__restrict__ W, int lane)
{
    constexpr int NB = 2 * NC;
    constexpr int NBF = NC / R;
    constexpr int PER = (NBF + kWave - 1) / kWave;   // butterflies per lane
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = p * kWave + lane;
        if (NBF % kWave == 0 || j < NBF) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if constexpr (FROM_INT) {
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
                constexpr int STRIDE = NB / (NS * R);
#pragma unroll
                for (int t = 1; t < R; ++t) v[p][t] = cmul(v[p][t], W[(t * k * STRIDE) & (NB - 1)]);
            }
            dftR<R>(v[p]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[swz(base + t * NS)] = v[p][t];
        }
    }
}

// In-place complex FFT of the NC = NB/2 packed points z_n = h_2n + i h_2n+1
// (radix 8 while possible, then 4 or 2); Z ends in natural order, swizzled.
template <int NC, int NS, bool FROM_INT>
__device__ __forceinline__ void fft_inplace(float2 *buf, const float2 *__restrict__ W, int lane)
{
    constexpr int REM = NC / NS;
    if constexpr (REM > 1) {
        constexpr int R = REM >= 8 ? 8 : REM;
        stockham_pass<NC, R, NS, FROM_INT>(buf, W, lane);
        wave_lds_sync();
        fft_inplace<NC, NS * R, false>(buf, W, lane);
    }
}

// |X_k| of the real input from the packed complex transform Z (length NC,
// swizzled): X_k = E_k + exp(-2 pi i k / NB) O_k, E_k = (Z_k + conj Z_{NC-k}) / 2,
// O_k = -i (Z_k - conj Z_{NC-k}) / 2, for 0 <= k <= NC.
template <int NC>
__device__ __forceinline__ float real_amplitude(const float2 *__restrict__ Z, const float2 *__restrict__ W, int k)
{
    const float2 zk = Z[swz(k & (NC - 1))];
    const float2 zm = Z[swz((NC - k) & (NC - 1))];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    const float2 x = cadd(e, cmul(W[k], o));
    return sqrtf(fmaf(x.x, x.x, x.y * x.y));
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
