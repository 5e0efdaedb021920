// Orientation refinement below the library grid with an unbinned
// structure-factor score built on the direct Fourier transform of Eq. (2)
// (Sec. 2.2, FSP paragraph), evaluated on spherical shells |k| = f_w along
// the mesh directions rotated by the ROI orientation q:
//   u_v = R(q/|q|) n_v,  F_{w,v} = sum_j exp(-2 pi i f_w u_v . x_j) = C - i S,
//   C = sum_j cos th_j, S = sum_j sin th_j, th_j = 2 pi f_w u_v . x_j,
//   A = |F| / N_w,  J = sum_{w,v} (A - T_{p,w,v})^2.
// Adjoint: with P = sum_j x_j sin th_j and Q = sum_j x_j cos th_j,
//   d|F|/du = 2 pi f (S Q - C P) / |F|,
//   dJ/du_v = sum_w 2 (A - T) / N_w * d|F|/du,
//   G = dJ/dR = sum_v (dJ/du_v) n_v^T,
//   dJ/dq^ = sum_ab G_ab dR_ab/dq^,   dJ/dq = (I - q^ q^T) dJ/dq^ / |q|.
//
// gfx950 design: one workgroup per (ROI, 256-direction tile); the ROI's
// relative coordinates are staged in LDS (broadcast reads: every lane of a
// wave reads the same atom), each lane owns one direction and all
// frequencies, sin/cos by the hardware transcendental unit (v_sin_f32 and
// v_cos_f32 take the phase in turns, so f * (u . x) needs no 2 pi and no
// range reduction for |f u.x| < 256).  Per-tile partial sums (J and the
// 3x3 G) are reduced across tiles in a fixed order by a second kernel, so
// results are deterministic.
//
// Antipodal pairs: F(-u) is the complex conjugate of F(u), so A(-u) = A(u).
// The geodesic mesh is centrally symmetric (n_v' = -n_v exactly), so each
// antipodal pair is evaluated once: with e = A - T_v and e' = A - T_v',
// J gains e^2 + e'^2 and the pair's gradient is (e + e') dA/du_v n_v^T
// (d/dR of A(R n_v') equals d/dR of A(R n_v) because A is even in u).
// Directions without an exact antipode are evaluated on their own.
#include <math.h>

#include <mutex>

#include "ar_internal.h"

namespace ar {
namespace sf {

constexpr int kTile = 256;       // directions per workgroup
constexpr int kMaxFreq = 8;
constexpr int kChunk = 1024;     // atoms staged in LDS per pass
constexpr int kPartial = 10;     // J + G(3x3)

template <typename T>
__device__ __forceinline__ void rotation(const T *q, T *M)
{
    T w = q[0], x = q[1], y = q[2], z = q[3];
    const T n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

// One evaluated direction v (antipode vm, or -1) from its sums: MODE 2 writes
// the amplitudes; otherwise J gains e^2 + e'^2 per frequency and, for MODE 1,
// gu the pair's dJ/du.
template <int MODE, int NF>
__device__ __forceinline__ void sf_direction(const float (&C)[NF], const float (&S)[NF], const float (&P)[NF][3],
                                             const float (&Q)[NF][3], const float (&f)[NF], int nw, bool valid,
                                             int v, int vm, int p, int n_dir, const float *__restrict__ targets,
                                             float *__restrict__ amp, int64_t r, float &J, float (&gu)[3])
{
    const float inv_n = nw > 0 ? 1.0f / (float)nw : 0.f;
#pragma unroll
    for (int w = 0; w < NF; ++w) {
        const float mag = sqrtf(fmaf(C[w], C[w], S[w] * S[w]));
        const float A = mag * inv_n;
        if (MODE == 2) {
            if (valid) {
                amp[((size_t)r * NF + w) * n_dir + v] = A;
                if (vm >= 0) amp[((size_t)r * NF + w) * n_dir + vm] = A;
            }
            continue;
        }
        const float e = valid ? A - targets[((size_t)p * NF + w) * n_dir + v] : 0.f;
        const float em = (valid && vm >= 0) ? A - targets[((size_t)p * NF + w) * n_dir + vm] : 0.f;
        J = fmaf(e, e, J);
        J = fmaf(em, em, J);
        if (MODE == 1 && valid && mag >= 1e-12f * (float)nw && nw > 0) {
            const float k = 2.0f * (e + em) * inv_n * 6.283185307179586f * f[w] / mag;
            gu[0] = fmaf(k, S[w] * Q[w][0] - C[w] * P[w][0], gu[0]);
            gu[1] = fmaf(k, S[w] * Q[w][1] - C[w] * P[w][1], gu[1]);
            gu[2] = fmaf(k, S[w] * Q[w][2] - C[w] * P[w][2], gu[2]);
        }
    }
}

constexpr int kRemAtoms = 16;   // a last tile with fewer directions runs atom-parallel

__device__ __forceinline__ void swap_acc(float &a, float &b)
{
    const float t = a;
    a = b;
    b = t;
}

// One atom's terms for one direction: the phases in turns, their sin and
// cos, and the C, S, P, Q sums.  (ax, ay, az) = f_kb u, so the dot product
// is slot 0's phase; slot w's is g_w = f / f_kb times it.
template <int MODE, int NF>
__device__ __forceinline__ void sf_term(const float4 x, float ax, float ay, float az, const float (&g)[NF],
                                        float (&C)[NF], float (&S)[NF], float (&P)[NF][3], float (&Q)[NF][3])
{
    const float d = fmaf(az, x.z, fmaf(ay, x.y, ax * x.x));
#pragma unroll
    for (int w = 0; w < NF; ++w) {
        const float t = w == 0 ? d : g[w] * d;   // phase in turns
        const float sn = __builtin_amdgcn_sinf(t);
        const float cs = __builtin_amdgcn_cosf(t);
        C[w] += cs;
        S[w] += sn;
        if (MODE == 1) {
            P[w][0] = fmaf(x.x, sn, P[w][0]);
            P[w][1] = fmaf(x.y, sn, P[w][1]);
            P[w][2] = fmaf(x.z, sn, P[w][2]);
            Q[w][0] = fmaf(x.x, cs, Q[w][0]);
            Q[w][1] = fmaf(x.y, cs, Q[w][1]);
            Q[w][2] = fmaf(x.z, cs, Q[w][2]);
        }
    }
}

// MODE 0: score partials; MODE 1: score + gradient partials; MODE 2: amplitudes.
// NF: number of frequencies (compile-time so the accumulators stay in VGPRs).
// A last tile with fewer than kRemAtoms directions (e.g. the one direction
// left after 20 full tiles of the 10242-node mesh's 5121 evaluated ones) is
// left to k_sf_rem, which splits the atoms over the threads instead, so that
// it costs a few atom passes rather than a full tile's.
template <int MODE, int NF>
__global__ __launch_bounds__(kTile) void k_sf(const float4 *__restrict__ rel, const int64_t *__restrict__ offsets,
                                              const float *__restrict__ quats, const int32_t *__restrict__ phase,
                                              int n_phase, const float *__restrict__ dirs, int n_dir,
                                              const int32_t *__restrict__ rep,
                                              const int32_t *__restrict__ mate, const int32_t *__restrict__ n_eval_p,
                                              int n_tiles, int64_t n_roi,
                                              const float *__restrict__ freqs, const float *__restrict__ targets,
                                              float *__restrict__ partials, float *__restrict__ amp)
{
    __shared__ float4 xs[kChunk];
    __shared__ float red[kPartial][kTile / 64];
    // XCD-aware order: workgroup ids go round-robin to the 8 XCDs; item t =
    // (b % 8) * (grid / 8) + b / 8 keeps the tiles of one ROI on one XCD, so
    // its atoms come from HBM into that XCD's L2 once (grid padded to 8)
    const int64_t t = (int64_t)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (t >= n_roi * n_tiles) return;
    const int64_t r = t / n_tiles;
    const int tile = (int)(t - r * n_tiles);
    const int n_eval = *n_eval_p;
    if (tile * kTile >= n_eval) {       // tiles past the evaluation list: nothing to add
        if (MODE != 2 && threadIdx.x < kPartial) partials[((size_t)r * n_tiles + tile) * kPartial + threadIdx.x] = 0.f;
        return;
    }
    const int i_eval = tile * kTile + threadIdx.x;
    const bool valid = i_eval < n_eval;
    const int v = valid ? rep[i_eval] : 0;
    const int vm = valid ? mate[i_eval] : -1;
    const int p = min(max(phase[r], 0), n_phase - 1);   // out-of-range phases are clamped
    float q[4] = {quats[4 * r], quats[4 * r + 1], quats[4 * r + 2], quats[4 * r + 3]};
    float M[9];
    rotation(q, M);
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (valid) {
        nx = dirs[3 * v];
        ny = dirs[3 * v + 1];
        nz = dirs[3 * v + 2];
    }
    const float ux = M[0] * nx + M[1] * ny + M[2] * nz;
    const float uy = M[3] * nx + M[4] * ny + M[5] * nz;
    const float uz = M[6] * nx + M[7] * ny + M[8] * nz;
    float f[NF];
#pragma unroll
    for (int w = 0; w < NF; ++w) f[w] = freqs[p * NF + w];
    // phases: the loop puts the frequency of largest |f| (index kb) in slot
    // 0 and forms its phase as one dot product with f_kb u; every other slot
    // w takes (f / f_kb) times it, one multiply per atom fewer than f (u . x)
    // per frequency, and |f / f_kb| <= 1 cannot overflow.  Slots 0 and kb
    // hold frequencies kb and 0; the sums go back to frequency order after
    // the loop.  All-zero frequencies give zero phases (g = 0, f_kb u = 0).
    int kb = 0;
#pragma unroll
    for (int w = 1; w < NF; ++w)
        if (fabsf(f[w]) > fabsf(f[kb])) kb = w;
    const float fb = f[kb];
    float g[NF];
#pragma unroll
    for (int w = 0; w < NF; ++w) {   // uniform over the workgroup: scalar registers
        const float fw = w == 0 ? fb : (w == kb ? f[0] : f[w]);
        const float gw = fb != 0.f ? fw / fb : 0.f;
        g[w] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, gw)));
    }
    const float ax = fb * ux, ay = fb * uy, az = fb * uz;
    float C[NF], S[NF], P[NF][3], Q[NF][3];
#pragma unroll
    for (int w = 0; w < NF; ++w) {
        C[w] = S[w] = 0.f;
        P[w][0] = P[w][1] = P[w][2] = Q[w][0] = Q[w][1] = Q[w][2] = 0.f;
    }
    const int64_t off0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - off0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (n_eval - tile * kTile < kRemAtoms) return;   // a short last tile: k_sf_rem writes it
    // a wave whose 64 directions all lie past the evaluation list (in the
    // last, partial tile) only helps stage the atoms
    const bool wave_busy = __builtin_amdgcn_readfirstlane(tile * kTile + (int)(threadIdx.x & ~63u)) < n_eval;
    for (int c0 = 0; c0 < nw; c0 += kChunk) {
        const int nc = min(kChunk, nw - c0);
        __syncthreads();
        // The fourth component is never read: setting it here lets the
        // staging load 12 bytes per atom instead of 16 (measured 3 % faster
        // per launch than copying the 16-byte rows).
        for (int i = threadIdx.x; i < nc; i += kTile) {
            float4 a = rel[off0 + c0 + i];
            a.w = 0.f;
            xs[i] = a;
        }
        __syncthreads();
        const int n_run = __builtin_amdgcn_readfirstlane(wave_busy ? nc : 0);
        // Two atoms per iteration with the schedule shaped by scheduling
        // groups (masks: 0x100 LDS read, 0x2 VALU, 0x400 transcendental):
        // both LDS reads, then per atom the dot product, a sin/cos pair,
        // the NF - 1 ratio multiplies, the other transcendentals and the
        // accumulations (8 NF with the gradient, else 2 NF).  Measured at
        // NF = 4 with the gradient against one atom per iteration (the best
        // unshaped form): 4 % faster.  Shapes that interleave each sin/cos
        // pair with accumulations, or take four atoms, measured 8 % and 5 %
        // slower than one atom per iteration.
        constexpr int kAcc = MODE == 1 ? 8 * NF : 2 * NF;
        int j = 0;
#pragma unroll 1
        for (; j + 1 < n_run; j += 2) {
            sf_term<MODE, NF>(xs[j], ax, ay, az, g, C, S, P, Q);
            sf_term<MODE, NF>(xs[j + 1], ax, ay, az, g, C, S, P, Q);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                __builtin_amdgcn_sched_group_barrier(0x2, 3, 0);
                __builtin_amdgcn_sched_group_barrier(0x400, 2, 0);
                if (NF > 1) {
                    __builtin_amdgcn_sched_group_barrier(0x2, NF - 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x400, 2 * NF - 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x2, kAcc, 0);
            }
        }
        if (j < n_run) sf_term<MODE, NF>(xs[j], ax, ay, az, g, C, S, P, Q);
    }
#pragma unroll
    for (int w = 1; w < NF; ++w) {   // slots back to frequency order
        if (w == kb) {
            swap_acc(C[0], C[w]);
            swap_acc(S[0], S[w]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                swap_acc(P[0][c], P[w][c]);
                swap_acc(Q[0][c], Q[w][c]);
            }
        }
    }
    float J = 0.f, gu[3] = {0.f, 0.f, 0.f};
    sf_direction<MODE, NF>(C, S, P, Q, f, nw, valid, v, vm, p, n_dir, targets, amp, r, J, gu);
    if (MODE == 2) return;
    float part[kPartial];
    part[0] = J;
    part[1] = gu[0] * nx; part[2] = gu[0] * ny; part[3] = gu[0] * nz;
    part[4] = gu[1] * nx; part[5] = gu[1] * ny; part[6] = gu[1] * nz;
    part[7] = gu[2] * nx; part[8] = gu[2] * ny; part[9] = gu[2] * nz;
#pragma unroll
    for (int k = 0; k < kPartial; ++k) {
        float x = part[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < kPartial) {
        float x = 0.f;
#pragma unroll
        for (int w = 0; w < kTile / 64; ++w) x += red[threadIdx.x][w];
        partials[((size_t)r * n_tiles + tile) * kPartial + threadIdx.x] = x;
    }
}

// The short last tile of each ROI (fewer than kRemAtoms evaluated
// directions left after the full tiles): one workgroup per ROI, each
// direction with the 256 threads split over the atoms (thread t sums atoms
// t, t + 256, ...), the block reducing the 8 NF sums (2 NF without the
// gradient); writes that tile's partials (or amplitudes).  Same arguments
// as k_sf.
template <int MODE, int NF>
__global__ __launch_bounds__(kTile) void k_sf_rem(const float4 *__restrict__ rel, const int64_t *__restrict__ offsets,
                                                  const float *__restrict__ quats, const int32_t *__restrict__ phase,
                                                  int n_phase, const float *__restrict__ dirs, int n_dir,
                                                  const int32_t *__restrict__ rep, const int32_t *__restrict__ mate,
                                                  const int32_t *__restrict__ n_eval_p, int n_tiles,
                                                  const float *__restrict__ freqs, const float *__restrict__ targets,
                                                  float *__restrict__ partials, float *__restrict__ amp)
{
    const int64_t r = blockIdx.x;
    const int n_eval = *n_eval_p;
    const int tile = n_eval / kTile;
    const int rem = n_eval - tile * kTile;
    if (rem == 0 || rem >= kRemAtoms) return;
    const int p = min(max(phase[r], 0), n_phase - 1);   // out-of-range phases are clamped
    float q[4] = {quats[4 * r], quats[4 * r + 1], quats[4 * r + 2], quats[4 * r + 3]};
    float M[9];
    rotation(q, M);
    float f[NF];
#pragma unroll
    for (int w = 0; w < NF; ++w) f[w] = freqs[p * NF + w];
    const int64_t off0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - off0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // atom-parallel: per direction, thread t sums atoms t, t + 256, ...,
    // then the block reduces the 8 NF sums (2 NF without the gradient)
    __shared__ float rs[8 * kMaxFreq][kTile / 64];
    constexpr int NV = MODE == 1 ? 8 * NF : 2 * NF;
    float Jt = 0.f, G[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int d = 0; d < rem; ++d) {
        const int vd = rep[tile * kTile + d], vmd = mate[tile * kTile + d];
        const float dx = dirs[3 * vd], dy = dirs[3 * vd + 1], dz = dirs[3 * vd + 2];
        const float wx = M[0] * dx + M[1] * dy + M[2] * dz;
        const float wy = M[3] * dx + M[4] * dy + M[5] * dz;
        const float wz = M[6] * dx + M[7] * dy + M[8] * dz;
        float acc[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = 0.f;
        for (int j = threadIdx.x; j < nw; j += kTile) {
            const float4 x = rel[off0 + j];
            const float sd = fmaf(wz, x.z, fmaf(wy, x.y, wx * x.x));
#pragma unroll
            for (int w = 0; w < NF; ++w) {
                const float t = f[w] * sd;
                const float sn = __builtin_amdgcn_sinf(t);
                const float cs = __builtin_amdgcn_cosf(t);
                acc[w] += cs;
                acc[NF + w] += sn;
                if (MODE == 1) {
                    acc[2 * NF + 3 * w] = fmaf(x.x, sn, acc[2 * NF + 3 * w]);
                    acc[2 * NF + 3 * w + 1] = fmaf(x.y, sn, acc[2 * NF + 3 * w + 1]);
                    acc[2 * NF + 3 * w + 2] = fmaf(x.z, sn, acc[2 * NF + 3 * w + 2]);
                    acc[5 * NF + 3 * w] = fmaf(x.x, cs, acc[5 * NF + 3 * w]);
                    acc[5 * NF + 3 * w + 1] = fmaf(x.y, cs, acc[5 * NF + 3 * w + 1]);
                    acc[5 * NF + 3 * w + 2] = fmaf(x.z, cs, acc[5 * NF + 3 * w + 2]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            float x = acc[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) rs[k][wave] = x;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float tot[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) tot[k] = rs[k][0] + rs[k][1] + rs[k][2] + rs[k][3];
            float Cd[NF], Sd[NF], Pd[NF][3], Qd[NF][3];
#pragma unroll
            for (int w = 0; w < NF; ++w) {
                Cd[w] = tot[w];
                Sd[w] = tot[NF + w];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Pd[w][c] = MODE == 1 ? tot[(2 * NF + 3 * w + c) % NV] : 0.f;
                    Qd[w][c] = MODE == 1 ? tot[(5 * NF + 3 * w + c) % NV] : 0.f;
                }
            }
            float gd[3] = {0.f, 0.f, 0.f};
            sf_direction<MODE, NF>(Cd, Sd, Pd, Qd, f, nw, true, vd, vmd, p, n_dir, targets, amp, r, Jt, gd);
            G[0] = fmaf(gd[0], dx, G[0]); G[1] = fmaf(gd[0], dy, G[1]); G[2] = fmaf(gd[0], dz, G[2]);
            G[3] = fmaf(gd[1], dx, G[3]); G[4] = fmaf(gd[1], dy, G[4]); G[5] = fmaf(gd[1], dz, G[5]);
            G[6] = fmaf(gd[2], dx, G[6]); G[7] = fmaf(gd[2], dy, G[7]); G[8] = fmaf(gd[2], dz, G[8]);
        }
        __syncthreads();
    }
    if (MODE != 2 && threadIdx.x == 0) {
        float *o = partials + ((size_t)r * n_tiles + tile) * kPartial;
        o[0] = Jt;
#pragma unroll
        for (int k = 0; k < 9; ++k) o[1 + k] = G[k];
    }
}

// Antipodal pairing of the directions.  mate_of[v] = the smallest u with
// n_u == -n_v exactly, else -1.  One thread per v, all u scanned (done once
// per call; the list is rebuilt on the device, nothing is cached by pointer).
__global__ __launch_bounds__(256) void k_antipodes(const float *__restrict__ dirs, int n_dir,
                                                   int32_t *__restrict__ mate_of)
{
    __shared__ float sd[3 * 256];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    float x = 0.f, y = 0.f, z = 0.f;
    if (v < n_dir) {
        x = -dirs[3 * v];
        y = -dirs[3 * v + 1];
        z = -dirs[3 * v + 2];
    }
    int found = -1;
    for (int u0 = 0; u0 < n_dir; u0 += 256) {
        __syncthreads();
        const int u = u0 + threadIdx.x;
        if (u < n_dir) {
            sd[3 * threadIdx.x] = dirs[3 * u];
            sd[3 * threadIdx.x + 1] = dirs[3 * u + 1];
            sd[3 * threadIdx.x + 2] = dirs[3 * u + 2];
        }
        __syncthreads();
        const int m = min(256, n_dir - u0);
        for (int k = 0; k < m; ++k)
            if (found < 0 && sd[3 * k] == x && sd[3 * k + 1] == y && sd[3 * k + 2] == z) found = u0 + k;
    }
    if (v < n_dir) mate_of[v] = found;
}

// Evaluation list: v is evaluated iff it has no antipode or its antipode has
// a larger index (then mate = antipode).  Written in index order by one
// workgroup with a block-wide prefix sum.
__global__ __launch_bounds__(1024) void k_eval_list(const int32_t *__restrict__ mate_of, int n_dir,
                                                    int32_t *__restrict__ rep, int32_t *__restrict__ mate,
                                                    int32_t *__restrict__ n_eval)
{
    __shared__ int32_t scan[1024];
    __shared__ int32_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int v0 = 0; v0 < n_dir; v0 += 1024) {
        const int v = v0 + threadIdx.x;
        int keep = 0, m = -1;
        if (v < n_dir) {
            m = mate_of[v];
            // pairs need mutual mates (n_v' = -n_v both ways); self-pairs cannot occur
            keep = (m < 0 || m > v) ? 1 : 0;
            if (m >= 0 && mate_of[m] != v) { keep = 1; m = -1; }
        }
        scan[threadIdx.x] = keep;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int t = threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += t;
            __syncthreads();
        }
        if (keep) {
            const int pos = base + scan[threadIdx.x] - 1;
            rep[pos] = v;
            mate[pos] = m;
        }
        __syncthreads();
        if (threadIdx.x == 1023) base += scan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_eval = base;
}

// dJ/dq from G for the normalised quaternion, projected on the tangent space.
__device__ __forceinline__ void grad_from_G(const float *q, const float *G, float *g)
{
    const float n = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    // dR/dw, dR/dx, dR/dy, dR/dz (row-major 3x3) of the rotation formula
    const float D[4][9] = {
        {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0}};
    float gh[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) a = fmaf(G[k], D[i][k], a);
        gh[i] = a;
    }
    const float qh[4] = {w, x, y, z};
    const float dot = gh[0] * w + gh[1] * x + gh[2] * y + gh[3] * z;
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = (gh[i] - qh[i] * dot) / n;
}

// Sum the tile partials of each ROI in tile order; write score (and grad).
__global__ __launch_bounds__(256) void k_sf_reduce(const float *__restrict__ partials, int n_tiles, int64_t n_roi,
                                                   const float *__restrict__ quats, float *__restrict__ score,
                                                   float *__restrict__ grad)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roi) return;
    float acc[kPartial];
#pragma unroll
    for (int k = 0; k < kPartial; ++k) acc[k] = 0.f;
    for (int t = 0; t < n_tiles; ++t)
#pragma unroll
        for (int k = 0; k < kPartial; ++k) acc[k] += partials[((size_t)r * n_tiles + t) * kPartial + k];
    if (score) score[r] = acc[0];
    if (grad) {
        const float q[4] = {quats[4 * r], quats[4 * r + 1], quats[4 * r + 2], quats[4 * r + 3]};
        float g[4];
        grad_from_G(q, acc + 1, g);
#pragma unroll
        for (int i = 0; i < 4; ++i) grad[4 * r + i] = g[i];
    }
}

// ------------------------------------------------------------ FP64 forward
__global__ __launch_bounds__(kTile) void k_sf_f64(const float4 *__restrict__ rel, const int64_t *__restrict__ offsets,
                                                  const double *__restrict__ quats, const int32_t *__restrict__ phase,
                                                  int n_phase, const float *__restrict__ dirs, int n_dir, int n_tiles,
                                                  const double *__restrict__ freqs, const double *__restrict__ targets,
                                                  int n_freq, double *__restrict__ partials)
{
    __shared__ float4 xs[kChunk];
    __shared__ double red[kTile / 64];
    const int64_t r = blockIdx.x / n_tiles;
    const int tile = blockIdx.x - (int)(r * n_tiles);
    const int v = tile * kTile + threadIdx.x;
    const bool valid = v < n_dir;
    const int p = min(max(phase[r], 0), n_phase - 1);   // out-of-range phases are clamped
    double q[4] = {quats[4 * r], quats[4 * r + 1], quats[4 * r + 2], quats[4 * r + 3]};
    double M[9];
    rotation(q, M);
    double nx = 0, ny = 0, nz = 0;
    if (valid) {
        nx = dirs[3 * v];
        ny = dirs[3 * v + 1];
        nz = dirs[3 * v + 2];
    }
    const double ux = M[0] * nx + M[1] * ny + M[2] * nz;
    const double uy = M[3] * nx + M[4] * ny + M[5] * nz;
    const double uz = M[6] * nx + M[7] * ny + M[8] * nz;
    double C[kMaxFreq], S[kMaxFreq];
    for (int w = 0; w < kMaxFreq; ++w) C[w] = S[w] = 0.0;
    const int64_t off0 = offsets[r];
    const int nw = (int)(offsets[r + 1] - off0);
    for (int c0 = 0; c0 < nw; c0 += kChunk) {
        const int nc = min(kChunk, nw - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < nc; i += kTile) xs[i] = rel[off0 + c0 + i];
        __syncthreads();
        for (int j = 0; j < nc; ++j) {
            const float4 x = xs[j];
            const double s = ux * (double)x.x + uy * (double)x.y + uz * (double)x.z;
            for (int w = 0; w < n_freq; ++w) {
                double sn, cs;
                sincospi(2.0 * freqs[p * n_freq + w] * s, &sn, &cs);
                C[w] += cs;
                S[w] += sn;
            }
        }
    }
    double J = 0.0;
    for (int w = 0; w < n_freq; ++w) {
        const double A = nw > 0 ? sqrt(C[w] * C[w] + S[w] * S[w]) / (double)nw : 0.0;
        const double e = valid ? A - targets[((size_t)p * n_freq + w) * n_dir + v] : 0.0;
        J += e * e;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) J += __shfl_xor(J, o);
    if (lane == 0) red[wave] = J;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0;
        for (int w = 0; w < kTile / 64; ++w) x += red[w];
        partials[(size_t)r * n_tiles + tile] = x;
    }
}

__global__ __launch_bounds__(256) void k_sf_reduce_f64(const double *__restrict__ partials, int n_tiles,
                                                       int64_t n_roi, double *__restrict__ score)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roi) return;
    double acc = 0.0;
    for (int t = 0; t < n_tiles; ++t) acc += partials[(size_t)r * n_tiles + t];
    score[r] = acc;
}

// ------------------------------------------------------------ refinement
struct RefineState {
    float q[4];      // accepted orientation
    float g[4];      // gradient at q
    float J;         // score at q
    float a;         // step length (radians of quaternion arc)
};

// Evaluations happen at the trial quaternions `trial`.  Step 0 only
// initialises the state from the first evaluation.  gt == nullptr: the
// evaluation took the score alone (the last one, whose gradient would only
// feed a trial that is never evaluated); an accepted trial then keeps the
// previous gradient, or zero at step 0.
__global__ __launch_bounds__(256) void k_refine_update(RefineState *__restrict__ st, float *__restrict__ trial,
                                                       const float *__restrict__ Jt, const float *__restrict__ gt,
                                                       int64_t n_roi, int first, float a0)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roi) return;
    RefineState s = st[r];
    if (first) {
        for (int i = 0; i < 4; ++i) {
            s.q[i] = trial[4 * r + i];
            s.g[i] = gt ? gt[4 * r + i] : 0.f;
        }
        s.J = Jt[r];
        s.a = a0;
    } else {
        const float gn = sqrtf(s.g[0] * s.g[0] + s.g[1] * s.g[1] + s.g[2] * s.g[2] + s.g[3] * s.g[3]);
        if (Jt[r] <= s.J - 1e-4f * s.a * gn) {
            for (int i = 0; i < 4; ++i) {
                s.q[i] = trial[4 * r + i];
                if (gt) s.g[i] = gt[4 * r + i];
            }
            s.J = Jt[r];
            s.a *= 1.5f;
        } else {
            s.a *= 0.5f;
        }
    }
    // next trial: q - a g/|g|, normalised (the current q when g = 0)
    const float gn = sqrtf(s.g[0] * s.g[0] + s.g[1] * s.g[1] + s.g[2] * s.g[2] + s.g[3] * s.g[3]);
    float t[4];
    const float k = gn > 0.f ? s.a / gn : 0.f;
    for (int i = 0; i < 4; ++i) t[i] = s.q[i] - k * s.g[i];
    const float tn = sqrtf(t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + t[3] * t[3]);
    for (int i = 0; i < 4; ++i) trial[4 * r + i] = t[i] / tn;
    st[r] = s;
}

__global__ __launch_bounds__(256) void k_refine_finish(const RefineState *__restrict__ st, int64_t n_roi,
                                                       float *__restrict__ quats, float *__restrict__ score)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roi) return;
    for (int i = 0; i < 4; ++i) quats[4 * r + i] = st[r].q[i];
    if (score) score[r] = st[r].J;
}

__global__ void k_copy4(const float *__restrict__ a, float *__restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4 * n) b[i] = a[i];
}

}  // namespace sf

static ar_status sf_check(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi, const void *quats,
                          const int32_t *phase, const float *dirs, int32_t n_dir, const void *freqs, int32_t n_phase,
                          int32_t n_freq)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(rel && offsets && quats && phase && dirs && freqs, "NULL argument");
    AR_CHECK(n_roi >= 1 && n_dir >= 1 && n_phase >= 1, "sizes must be >= 1");
    AR_CHECK(n_freq >= 1 && n_freq <= sf::kMaxFreq, "n_freq must be in [1, %d]", sf::kMaxFreq);
    const int64_t tiles = (n_dir + sf::kTile - 1) / sf::kTile;
    AR_CHECK(n_roi * tiles + 7 < (int64_t)INT32_MAX, "too many workgroups");
    return AR_OK;
}

using SfFn = void (*)(const float4 *, const int64_t *, const float *, const int32_t *, int, const float *, int,
                     const int32_t *, const int32_t *, const int32_t *, int, int64_t, const float *, const float *,
                     float *, float *);
using SfRemFn = void (*)(const float4 *, const int64_t *, const float *, const int32_t *, int, const float *, int,
                        const int32_t *, const int32_t *, const int32_t *, int, const float *, const float *, float *,
                        float *);

// Device evaluation list for `dirs` written to `base` (int32 [3 n_dir + 1]):
// mate_of, rep, mate [n_dir] each, then n_eval.
static size_t eval_list_ints(int32_t n_dir) { return 3 * (size_t)n_dir + 1; }

static ar_status eval_list_into(int32_t *base, const float *dirs, int32_t n_dir, hipStream_t s)
{
    int32_t *mate_of = base, *r = base + n_dir, *m = base + 2 * n_dir, *n = base + 3 * n_dir;
    sf::k_antipodes<<<(unsigned)((n_dir + 255) / 256), 256, 0, s>>>(dirs, n_dir, mate_of);
    AR_HIP(hipGetLastError());
    sf::k_eval_list<<<1, 1024, 0, s>>>(mate_of, n_dir, r, m, n);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

// The evaluation list in the context's workspace.
static ar_status eval_list(ar_context *ctx, const float *dirs, int32_t n_dir, hipStream_t s)
{
    AR_TRY(ctx->r_dirs.reserve(sizeof(int32_t) * eval_list_ints(n_dir)));
    return eval_list_into(ctx->r_dirs.as<int32_t>(), dirs, n_dir, s);
}

static size_t partial_floats(int64_t n_roi, int32_t n_dir)
{
    return (size_t)n_roi * ((n_dir + sf::kTile - 1) / sf::kTile) * sf::kPartial;
}

template <int MODE> SfFn sf_kernel(int n_freq)
{
    switch (n_freq) {
    case 1: return sf::k_sf<MODE, 1>;
    case 2: return sf::k_sf<MODE, 2>;
    case 3: return sf::k_sf<MODE, 3>;
    case 4: return sf::k_sf<MODE, 4>;
    case 5: return sf::k_sf<MODE, 5>;
    case 6: return sf::k_sf<MODE, 6>;
    case 7: return sf::k_sf<MODE, 7>;
    default: return sf::k_sf<MODE, 8>;
    }
}

template <int MODE> SfRemFn sf_rem_kernel(int n_freq)
{
    switch (n_freq) {
    case 1: return sf::k_sf_rem<MODE, 1>;
    case 2: return sf::k_sf_rem<MODE, 2>;
    case 3: return sf::k_sf_rem<MODE, 3>;
    case 4: return sf::k_sf_rem<MODE, 4>;
    case 5: return sf::k_sf_rem<MODE, 5>;
    case 6: return sf::k_sf_rem<MODE, 6>;
    case 7: return sf::k_sf_rem<MODE, 7>;
    default: return sf::k_sf_rem<MODE, 8>;
    }
}

// Launches of one evaluation with explicit workspace: `list` holds the
// evaluation list of eval_list_into, `part` (mode 0 and 1) the per-tile
// partials, float [n_roi][n_tiles][kPartial]; every partial is written before
// it is read, so neither needs clearing.
static ar_status sf_launch_ws(int mode, const float *rel, const int64_t *offsets, int64_t n_roi, const float *quats,
                              const int32_t *phase, int32_t n_phase, const float *dirs, int32_t n_dir,
                              const float *freqs, const float *targets, int32_t n_freq, float *score, float *grad,
                              float *amp, const int32_t *list, float *part, hipStream_t s)
{
    const int32_t *rep = list + n_dir, *mate = list + 2 * n_dir, *n_eval = list + 3 * n_dir;
    const int n_tiles = (n_dir + sf::kTile - 1) / sf::kTile;
    const unsigned blocks = (unsigned)((n_roi * n_tiles + 7) / 8 * 8);   // k_sf: a multiple of the 8 XCDs
    if (mode == 2) {
        sf_kernel<2>(n_freq)<<<blocks, sf::kTile, 0, s>>>((const float4 *)rel, offsets, quats, phase, n_phase, dirs, n_dir,
                                                          rep, mate, n_eval, n_tiles, n_roi, freqs, targets, nullptr,
                                                          amp);
        AR_HIP(hipGetLastError());
        sf_rem_kernel<2>(n_freq)<<<(unsigned)n_roi, sf::kTile, 0, s>>>((const float4 *)rel, offsets, quats, phase,
                                                                       n_phase, dirs, n_dir, rep, mate, n_eval, n_tiles,
                                                                       freqs, targets, nullptr, amp);
        AR_HIP(hipGetLastError());
        return AR_OK;
    }
    SfFn fn = mode == 1 ? sf_kernel<1>(n_freq) : sf_kernel<0>(n_freq);
    fn<<<blocks, sf::kTile, 0, s>>>((const float4 *)rel, offsets, quats, phase, n_phase, dirs, n_dir, rep, mate, n_eval,
                                    n_tiles, n_roi, freqs, targets, part, nullptr);
    AR_HIP(hipGetLastError());
    SfRemFn fr = mode == 1 ? sf_rem_kernel<1>(n_freq) : sf_rem_kernel<0>(n_freq);
    fr<<<(unsigned)n_roi, sf::kTile, 0, s>>>((const float4 *)rel, offsets, quats, phase, n_phase, dirs, n_dir, rep, mate,
                                             n_eval, n_tiles, freqs, targets, part, nullptr);
    AR_HIP(hipGetLastError());
    sf::k_sf_reduce<<<(unsigned)((n_roi + 255) / 256), 256, 0, s>>>(part, n_tiles, n_roi, quats, score,
                                                                    mode == 1 ? grad : nullptr);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

// One evaluation with the context's (growable) workspace.
static ar_status sf_launch(ar_context *ctx, int mode, const float *rel, const int64_t *offsets, int64_t n_roi,
                           const float *quats, const int32_t *phase, int32_t n_phase, const float *dirs,
                           int32_t n_dir, const float *freqs, const float *targets, int32_t n_freq, float *score,
                           float *grad, float *amp, hipStream_t s, bool have_list = false)
{
    if (!have_list) AR_TRY(eval_list(ctx, dirs, n_dir, s));
    float *part = nullptr;
    if (mode != 2) {
        AR_TRY(ctx->r_partials.reserve(sizeof(float) * partial_floats(n_roi, n_dir)));
        part = ctx->r_partials.as<float>();
    }
    return sf_launch_ws(mode, rel, offsets, n_roi, quats, phase, n_phase, dirs, n_dir, freqs, targets, n_freq, score,
                        grad, amp, ctx->r_dirs.as<int32_t>(), part, s);
}

// ---------------------------------------------- allocation-free workspace
// One fixed workspace per GPU for ar_sf_score_grad_noalloc: the evaluation
// list (256-byte aligned), then the per-tile partials.  It lives as long as
// the process; its device address is looked up once per device when a
// context is created on it (the array's name is not a device address in
// host code).
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch[kScratchDevices];
static std::mutex g_scratch_mu;

static size_t scratch_list_bytes(int32_t n_dir) { return (sizeof(int32_t) * eval_list_ints(n_dir) + 255) / 256 * 256; }

// Called by ar_context_create with `device` current.
ar_status scratch_setup(int device)
{
    if (device < 0 || device >= kScratchDevices) return AR_OK;   // the allocation-free call then refuses
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return AR_OK;
    void *p = nullptr;
    AR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    AR_CHECK(p != nullptr, "no device address for the fixed workspace on device %d", device);
    g_scratch[device] = p;
    return AR_OK;
}

}  // namespace ar

extern "C" {

ar_status ar_sf_score_grad(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                           const float *quats, const int32_t *phase, const float *directions, int32_t n_dir,
                           const float *freqs, const float *targets, int32_t n_phase, int32_t n_freq, float *score,
                           float *grad, void *stream)
{
    AR_TRY(ar::sf_check(ctx, rel, offsets, n_roi, quats, phase, directions, n_dir, freqs, n_phase, n_freq));
    AR_CHECK(targets && score, "targets/score must not be NULL");
    AR_HIP(hipSetDevice(ctx->device));
    return ar::sf_launch(ctx, grad ? 1 : 0, rel, offsets, n_roi, quats, phase, n_phase, directions, n_dir, freqs, targets,
                         n_freq, score, grad, nullptr, (hipStream_t)stream);
}

ar_status ar_sf_score_grad_noalloc(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                                   const float *quats, const int32_t *phase, const float *directions, int32_t n_dir,
                                   const float *freqs, const float *targets, int32_t n_phase, int32_t n_freq,
                                   float *score, float *grad, void *stream)
{
    AR_TRY(ar::sf_check(ctx, rel, offsets, n_roi, quats, phase, directions, n_dir, freqs, n_phase, n_freq));
    AR_CHECK(targets && score, "targets/score must not be NULL");
    const size_t list = ar::scratch_list_bytes(n_dir);
    const size_t need = list + sizeof(float) * ar::partial_floats(n_roi, n_dir);
    AR_CHECK(need <= ar::kScratchBytes,
             "n_roi = %lld and n_dir = %d need %zu bytes of workspace; the fixed workspace holds %zu "
             "(n_roi * ceil(n_dir / 256) * 40 + 12 n_dir bytes, about)",
             (long long)n_roi, n_dir, need, ar::kScratchBytes);
    AR_CHECK(ctx->device < ar::kScratchDevices, "device %d has no fixed workspace", ctx->device);
    unsigned char *base;
    {
        std::lock_guard<std::mutex> lock(ar::g_scratch_mu);
        base = static_cast<unsigned char *>(ar::g_scratch[ctx->device]);
    }
    AR_CHECK(base != nullptr, "fixed workspace of device %d not set up", ctx->device);
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int32_t *lst = reinterpret_cast<int32_t *>(base);
    float *part = reinterpret_cast<float *>(base + list);
    AR_TRY(ar::eval_list_into(lst, directions, n_dir, s));
    return ar::sf_launch_ws(grad ? 1 : 0, rel, offsets, n_roi, quats, phase, n_phase, directions, n_dir, freqs,
                            targets, n_freq, score, grad, nullptr, lst, part, s);
}

ar_status ar_sf_amplitudes(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                           const float *quats, const int32_t *phase, const float *directions, int32_t n_dir,
                           const float *freqs, int32_t n_phase, int32_t n_freq, float *amp, void *stream)
{
    AR_TRY(ar::sf_check(ctx, rel, offsets, n_roi, quats, phase, directions, n_dir, freqs, n_phase, n_freq));
    AR_CHECK(amp != nullptr, "amp is NULL");
    AR_HIP(hipSetDevice(ctx->device));
    return ar::sf_launch(ctx, 2, rel, offsets, n_roi, quats, phase, n_phase, directions, n_dir, freqs, nullptr, n_freq, nullptr,
                         nullptr, amp, (hipStream_t)stream);
}

ar_status ar_sf_score_f64(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                          const double *quats, const int32_t *phase, const float *directions, int32_t n_dir,
                          const double *freqs, const double *targets, int32_t n_phase, int32_t n_freq, double *score,
                          void *stream)
{
    AR_TRY(ar::sf_check(ctx, rel, offsets, n_roi, quats, phase, directions, n_dir, freqs, n_phase, n_freq));
    AR_CHECK(targets && score, "targets/score must not be NULL");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int n_tiles = (n_dir + ar::sf::kTile - 1) / ar::sf::kTile;
    AR_TRY(ctx->r_partials.reserve(sizeof(double) * (size_t)n_roi * n_tiles));
    double *part = ctx->r_partials.as<double>();
    ar::sf::k_sf_f64<<<(unsigned)(n_roi * n_tiles), ar::sf::kTile, 0, s>>>(
        (const float4 *)rel, offsets, quats, phase, n_phase, directions, n_dir, n_tiles, freqs, targets, n_freq, part);
    AR_HIP(hipGetLastError());
    ar::sf::k_sf_reduce_f64<<<(unsigned)((n_roi + 255) / 256), 256, 0, s>>>(part, n_tiles, n_roi, score);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

ar_status ar_refine_orientations(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                                 float *quats, const int32_t *phase, const float *directions, int32_t n_dir,
                                 const float *freqs, const float *targets, int32_t n_phase, int32_t n_freq,
                                 int32_t steps, float a0, float *score, void *stream)
{
    AR_TRY(ar::sf_check(ctx, rel, offsets, n_roi, quats, phase, directions, n_dir, freqs, n_phase, n_freq));
    AR_CHECK(targets != nullptr, "targets is NULL");
    AR_CHECK(steps >= 0 && steps <= 100000, "steps out of range");
    AR_CHECK(a0 > 0.f && isfinite(a0), "a0 must be finite and > 0");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // workspace: state, trial quaternions, trial score, trial gradient
    const size_t st_bytes = sizeof(ar::sf::RefineState) * n_roi;
    AR_TRY(ctx->r_state.reserve(st_bytes + sizeof(float) * 9 * n_roi + 256));
    char *base = ctx->r_state.as<char>();
    auto *st = reinterpret_cast<ar::sf::RefineState *>(base);
    float *trial = reinterpret_cast<float *>(base + ((st_bytes + 255) / 256) * 256);
    float *Jt = trial + 4 * n_roi;
    float *gt = Jt + n_roi;
    const unsigned nb = (unsigned)((n_roi + 255) / 256);
    ar::sf::k_copy4<<<(unsigned)((4 * n_roi + 255) / 256), 256, 0, s>>>(quats, trial, n_roi);
    AR_HIP(hipGetLastError());
    AR_TRY(ar::eval_list(ctx, directions, n_dir, s));
    for (int it = 0; it <= steps; ++it) {
        // the last evaluation only decides whether its trial is accepted:
        // score alone (the forward kernel, about half the adjoint's work)
        const bool last = it == steps;
        AR_TRY(ar::sf_launch(ctx, last ? 0 : 1, rel, offsets, n_roi, trial, phase, n_phase, directions, n_dir, freqs, targets,
                             n_freq, Jt, gt, nullptr, s, true));
        ar::sf::k_refine_update<<<nb, 256, 0, s>>>(st, trial, Jt, last ? nullptr : gt, n_roi, it == 0 ? 1 : 0, a0);
        AR_HIP(hipGetLastError());
    }
    ar::sf::k_refine_finish<<<nb, 256, 0, s>>>(st, n_roi, quats, score);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // extern "C"
