// Sparse orientation indexing: Eq. S1 evaluated at the strongest reference
// entries through a look-up table of rotated nodes (supplement, "Indexing
// algorithm"; creation cost O_lu = N_c N_g N^_v and indexing cost
// O_idx = N_roi N_c N_g N^_v of the complexity paragraph).
//
// Look-up table (ar_sparse_lut_create), per phase c:
//   1. k_ref_max        per window, the maximum of the raw reference image.
//   2. k_strong_rank    every entry's key x / max in FP64; its rank among all
//                       entries (larger key first, equal keys by lower flat
//                       index w * n_dir + v) by counting; ranks < n_hat are
//                       the strong entries in decreasing order.
//   3. k_window_order   the strong entries regrouped by window (stable), the
//                       order the screen kernel walks them in, with their
//                       values as FP16 pairs.
//   4. k_sparse_lut     for every orientation g of phase c and strong entry i:
//                       the mesh node closest to R(q_g) n_{v_i}.
//   5. k_lut_rows       the same table transposed to one row per orientation.
//
// Indexing (index_orientations_sparse):
//   1. k_sparse_norm    per (ROI, window) 1 / max in FP32; the normalised
//                       image in FP16, RB ROIs interleaved per node.
//   2. k_sparse_screen  one workgroup per (orientation chunk, group of RB
//                       ROIs): for each window, the RB ROI images of that
//                       window sit in LDS (RB FP16 values per node, one
//                       8/4/2-byte read per look-up); every lane owns four
//                       orientations, reads their look-up nodes (one 8-byte
//                       load per strong entry), forms s - R in packed FP16
//                       and accumulates the squares in FP32.  The
//                       workgroup keeps the CAND best orientations per ROI
//                       (per-wave selection, then a merge in LDS).
//   3. k_sparse_merge   per ROI, the CAND best over all chunks.
//   4. k_sparse_rescore exact FP32 Eq. S1 for the CAND candidates from the
//                       FP32 image; sorted by (Delta, index).
#include <math.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ar_internal.h"
#include "mesh_device.h"
#include "topk_device.h"

struct ar_sparse_lut {
    ar_context *ctx = nullptr;
    int32_t n_phase = 0, n_win = 0, n_dir = 0, n_hat = 0;
    int64_t n_lib = 0;
    int64_t ld = 0;                      // row length of lut_ig (orientations + padding)
    int32_t n_chunks = 0;
    ar::DeviceBuffer phase_start;        // int64 [n_phase + 1]
    ar::DeviceBuffer strong_idx;         // int32 [n_phase][n_hat], w * n_dir + v, decreasing value
    ar::DeviceBuffer strong_val;         // float [n_phase][n_hat], normalised value
    ar::DeviceBuffer kpos;               // int32 [n_phase][n_hat], position of entry i in window order
    ar::DeviceBuffer kval2;              // uint32 [n_phase][n_hat]: (R, R) in FP16, window order
    ar::DeviceBuffer seg;                // int32 [n_phase][n_win + 1], window segments of the window order
    ar::DeviceBuffer lut_ig;             // uint16 [n_hat][ld], window order of each column's phase
    ar::DeviceBuffer lut_gi;             // uint16 [n_lib][n_hat], decreasing-value order
    ar::DeviceBuffer chunks;             // int4 [n_chunks]: phase, first column (multiple of 4), valid [lo, hi)
};

namespace ar {
namespace sparse {

constexpr int kThreads = 1024;               // screen workgroup: 16 waves
constexpr int kWaves = kThreads / 64;
constexpr int kPerLane = 4;                  // orientations per lane
constexpr int kChunk = kPerLane * kThreads;  // orientations per workgroup

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ look-up table
__global__ __launch_bounds__(256) void k_ref_max(const float *__restrict__ ref, int n_dir, float *__restrict__ out)
{
    __shared__ float red[256];
    const float *src = ref + (size_t)blockIdx.x * n_dir;
    float m = 0.0f;
    for (int v = threadIdx.x; v < n_dir; v += 256) m = fmaxf(m, src[v]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// grid (ceil(K / 256), n_phase)
__global__ __launch_bounds__(256) void k_strong_rank(const float *__restrict__ ref, const float *__restrict__ ref_max,
                                                     int n_win, int n_dir, int n_hat, int32_t *__restrict__ strong_idx,
                                                     float *__restrict__ strong_val)
{
    __shared__ double tile[256];
    const int c = blockIdx.y;
    const int64_t K = (int64_t)n_win * n_dir;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float *img = ref + (size_t)c * K;
    const float *mx = ref_max + (size_t)c * n_win;
    auto key = [&](int64_t j) -> double {
        const float m = mx[j / n_dir];
        return m > 0.0f ? (double)img[j] / (double)m : 0.0;
    };
    const double mine = e < K ? key(e) : 0.0;
    int64_t rank = 0;
    for (int64_t t0 = 0; t0 < K; t0 += 256) {
        __syncthreads();
        if (t0 + threadIdx.x < K) tile[threadIdx.x] = key(t0 + threadIdx.x);
        __syncthreads();
        const int n = (int)min((int64_t)256, K - t0);
        for (int j = 0; j < n; ++j) {
            const double o = tile[j];
            rank += (o > mine || (o == mine && t0 + j < e)) ? 1 : 0;
        }
    }
    if (e < K && rank < n_hat) {
        strong_idx[(size_t)c * n_hat + rank] = (int32_t)e;
        strong_val[(size_t)c * n_hat + rank] = (float)mine;
    }
}

// grid (ceil(n_hat / 256), n_phase): window order = stable regrouping of the
// strong entries by window; seg[c][w] = number of strong entries in windows
// below w.
__global__ __launch_bounds__(256) void k_window_order(const int32_t *__restrict__ strong_idx,
                                                      const float *__restrict__ strong_val, int n_hat, int n_win,
                                                      int n_dir, int32_t *__restrict__ kpos, uint32_t *__restrict__ kval2,
                                                      int32_t *__restrict__ seg)
{
    const int c = blockIdx.y;
    const int32_t *si = strong_idx + (size_t)c * n_hat;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_hat) {
        const int wi = si[i] / n_dir;
        int pos = 0;
        for (int j = 0; j < n_hat; ++j) {
            const int wj = si[j] / n_dir;
            pos += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
        }
        kpos[(size_t)c * n_hat + i] = pos;
        const _Float16 h = (_Float16)strong_val[(size_t)c * n_hat + i];
        kval2[(size_t)c * n_hat + pos] = __builtin_bit_cast(uint32_t, half2_t{h, h});
    }
    if (blockIdx.x == 0)
        for (int w = threadIdx.x; w <= n_win; w += 256) {
            int cnt = 0;
            for (int j = 0; j < n_hat; ++j) cnt += (si[j] / n_dir < w) ? 1 : 0;
            seg[(size_t)c * (n_win + 1) + w] = cnt;
        }
}

__device__ __forceinline__ int phase_of(int64_t g, const int64_t *__restrict__ phase_start, int n_phase)
{
    int c = 0;
    while (c + 1 < n_phase && g >= phase_start[c + 1]) ++c;
    return c;
}

// grid (ceil(n_lib / 256), n_hat): one thread per (orientation, strong entry)
__global__ __launch_bounds__(256) void k_sparse_lut(const double *__restrict__ quats,
                                                    const int64_t *__restrict__ phase_start, int n_phase,
                                                    int64_t n_lib, const int32_t *__restrict__ strong_idx,
                                                    const int32_t *__restrict__ kpos, int n_hat,
                                                    const float *__restrict__ dirs, int n_dir,
                                                    uint16_t *__restrict__ lut_ig, int64_t ld)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y;
    const bool valid = g < n_lib;
    const int c = valid ? phase_of(g, phase_start, n_phase) : 0;
    const int v = strong_idx[(size_t)c * n_hat + i] % n_dir;
    double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (valid) quat_matrix64(quats + 4 * g, M);
    const double nx = dirs[3 * v], ny = dirs[3 * v + 1], nz = dirs[3 * v + 2];
    // R(q) n
    const double rx = M[0] * nx + M[1] * ny + M[2] * nz;
    const double ry = M[3] * nx + M[4] * ny + M[5] * nz;
    const double rz = M[6] * nx + M[7] * ny + M[8] * nz;
    const int p = nearest_node(rx, ry, rz, dirs, n_dir);
    if (valid) lut_ig[(size_t)kpos[(size_t)c * n_hat + i] * ld + g] = (uint16_t)p;
}

// one thread per (orientation, entry in decreasing-value order)
__global__ __launch_bounds__(256) void k_lut_rows(const uint16_t *__restrict__ lut_ig, int64_t ld,
                                                  const int32_t *__restrict__ kpos,
                                                  const int64_t *__restrict__ phase_start, int n_phase,
                                                  int64_t n_lib, int n_hat, uint16_t *__restrict__ lut_gi)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_lib * n_hat) return;
    const int64_t g = t / n_hat;
    const int i = (int)(t - g * n_hat);
    const int c = phase_of(g, phase_start, n_phase);
    lut_gi[t] = lut_ig[(size_t)kpos[(size_t)c * n_hat + i] * ld + g];
}

__global__ __launch_bounds__(256) void k_lut_export(const uint16_t *__restrict__ lut_gi, int64_t n,
                                                    int32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) out[t] = lut_gi[t];
}

// ------------------------------------------------------------ indexing
// The screen kernel addresses its window slab by integer LDS address from 0:
// it declares no static LDS, so its dynamic allocation is [0, bytes).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T *lds_at(uint32_t byte_offset)
{
    return (__attribute__((address_space(3))) T *)(size_t)byte_offset;
}

// Byte offset (node id << SHIFT) of the 16-bit node id in half H of a packed
// pair: one v_lshlrev_b32 with a word-select source operand.
template <int SHIFT, int H>
__device__ __forceinline__ uint32_t node_offset(uint32_t pair)
{
    uint32_t off;
    if (H == 0)
        asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
            : "=v"(off) : "v"(pair), "n"(SHIFT));
    else
        asm("v_lshlrev_b32_sdwa %0, %2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
            : "=v"(off) : "v"(pair), "n"(SHIFT));
    return off;
}

// acc[j] += (x_j - R)^2 for the RB FP16 values x at LDS byte offset `off`:
// the difference in packed FP16 (v_pk_add_f16), the square accumulated in
// FP32 (v_fma_mix_f32).  R2 holds (R, R) in FP16.
template <int RB>
struct RoiVec;
template <>
struct RoiVec<4> {
    static constexpr int SHIFT = 3;
    __device__ __forceinline__ static void acc(uint32_t off, uint32_t R2, float (&a)[4])
    {
        const half4_t x = *lds_at<const half4_t>(off);
        const half2_t R = __builtin_bit_cast(half2_t, R2);
        const half2_t d01 = x.xy - R, d23 = x.zw - R;
        a[0] = fmaf((float)d01.x, (float)d01.x, a[0]);
        a[1] = fmaf((float)d01.y, (float)d01.y, a[1]);
        a[2] = fmaf((float)d23.x, (float)d23.x, a[2]);
        a[3] = fmaf((float)d23.y, (float)d23.y, a[3]);
    }
};
template <>
struct RoiVec<2> {
    static constexpr int SHIFT = 2;
    __device__ __forceinline__ static void acc(uint32_t off, uint32_t R2, float (&a)[2])
    {
        const half2_t d = *lds_at<const half2_t>(off) - __builtin_bit_cast(half2_t, R2);
        a[0] = fmaf((float)d.x, (float)d.x, a[0]);
        a[1] = fmaf((float)d.y, (float)d.y, a[1]);
    }
};
template <>
struct RoiVec<1> {
    static constexpr int SHIFT = 1;
    __device__ __forceinline__ static void acc(uint32_t off, uint32_t R2, float (&a)[1])
    {
        const _Float16 d = *lds_at<const _Float16>(off) - __builtin_bit_cast(half2_t, R2).x;
        a[0] = fmaf((float)d, (float)d, a[0]);
    }
};

// grid (n_grp, n_win).  inv_s[r][w] = 1 / max (0 for an all-zero window);
// half[grp][w][slab]: node v of ROI grp * RB + j at half index v * RB + j
// (ROIs past n_roi and the slab padding are zero).
template <int RB>
__global__ __launch_bounds__(256) void k_sparse_norm(const float *__restrict__ img, int64_t n_roi, int n_win, int n_dir,
                                                     int64_t slab, float *__restrict__ inv_s,
                                                     _Float16 *__restrict__ half)
{
    __shared__ float red[256];
    __shared__ float inv[RB];
    const int64_t grp = blockIdx.x;
    const int w = blockIdx.y;
    for (int j = 0; j < RB; ++j) {
        const int64_t r = grp * RB + j;
        float m = 0.0f;
        if (r < n_roi) {
            const float *src = img + ((size_t)r * n_win + w) * n_dir;
            for (int v = threadIdx.x; v < n_dir; v += 256) m = fmaxf(m, src[v]);
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const float mx = red[0];
            inv[j] = mx > 0.0f ? 1.0f / mx : 0.0f;
            if (r < n_roi) inv_s[(size_t)r * n_win + w] = inv[j];
        }
        __syncthreads();
    }
    _Float16 *dst = half + ((size_t)grp * n_win + w) * slab;
    for (int64_t t = threadIdx.x; t < slab; t += 256) {
        const int v = (int)(t / RB), j = (int)(t - (int64_t)v * RB);
        const int64_t r = grp * RB + j;
        float x = 0.0f;
        if (v < n_dir && r < n_roi) x = img[((size_t)r * n_win + w) * n_dir + v] * inv[j];
        dst[t] = (_Float16)x;
    }
}

// grid: the (chunk, ROI group) work items padded to a multiple of 8; item t
// runs on XCD t / (grid / 8), so the 32 compute units of an XCD share the
// look-up rows of one chunk in their L2.
// out_s/out_i: [n_grp * RB][n_chunks][CAND]
template <int RB, int CAND>
__global__ __launch_bounds__(kThreads) void k_sparse_screen(
    const _Float16 *__restrict__ half, int n_win, int64_t slab, const uint16_t *__restrict__ lut_ig, int64_t ld,
    const uint32_t *__restrict__ kval2, const int32_t *__restrict__ seg, int n_hat, const int4 *__restrict__ chunks,
    int n_chunks, int n_grp, int64_t n_work, float *__restrict__ out_s, int32_t *__restrict__ out_i)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t nb8 = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (t >= n_work) return;
    const int chunk = (int)(t / n_grp);
    const int grp = (int)(t - (int64_t)chunk * n_grp);
    const int4 ch = chunks[chunk];
    const int tid = threadIdx.x;
    // each lane owns orientations ch.y + 4 tid .. + 3: one 8-byte load of
    // their four node ids per strong entry from a wave-uniform row address
    const uint16_t *lut_c = lut_ig + ch.y;
    const unsigned utid = threadIdx.x;
    const uint32_t *kv2 = kval2 + (size_t)ch.x * n_hat;
    const int32_t *sg = seg + (size_t)ch.x * (n_win + 1);

    float acc[kPerLane][RB];
#pragma unroll
    for (int g = 0; g < kPerLane; ++g)
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[g][r] = 0.0f;

    constexpr int SH = RoiVec<RB>::SHIFT;
    auto term = [&](uint2 pr, uint32_t R2) {
        RoiVec<RB>::acc(node_offset<SH, 0>(pr.x), R2, acc[0]);
        RoiVec<RB>::acc(node_offset<SH, 1>(pr.x), R2, acc[1]);
        RoiVec<RB>::acc(node_offset<SH, 0>(pr.y), R2, acc[2]);
        RoiVec<RB>::acc(node_offset<SH, 1>(pr.y), R2, acc[3]);
    };

    for (int w = 0; w < n_win; ++w) {
        const int j0 = sg[w], j1 = sg[w + 1];
        if (j0 == j1) continue;
        __syncthreads();   // every wave is done with the previous window
        {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(half + ((size_t)grp * n_win + w) * slab);
            const int n16 = (int)(slab >> 3);
            for (int q = tid; q < n16; q += kThreads) *lds_at<u32x4>(16u * q) = src[q];
        }
        __syncthreads();
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
            uint2 pr[4];
            uint32_t R2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pr[u] = reinterpret_cast<const uint2 *>(lut_c + (size_t)(j + u) * ld)[utid];
                R2[u] = kv2[j + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) term(pr[u], R2[u]);
        }
        for (; j < j1; ++j) term(reinterpret_cast<const uint2 *>(lut_c + (size_t)j * ld)[utid], kv2[j]);
    }

    // ---- the CAND best orientations of this chunk per ROI
    const int wave = tid >> 6, lane = tid & 63;
    __syncthreads();   // LDS now holds the wave lists
    float *ws = reinterpret_cast<float *>(smem);
    int32_t *wi = reinterpret_cast<int32_t *>(smem + sizeof(float) * kWaves * RB * CAND);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        TopList<kPerLane> tl;
        tl.init();
#pragma unroll
        for (int g = 0; g < kPerLane; ++g) {
            const int gi = ch.y + kPerLane * tid + g;
            if (gi >= ch.z && gi < ch.w) tl.insert(acc[g][r], gi);
        }
        wave_select<CAND>(tl, [&](int j, float bs, int bi) {
            if (lane == 0) {
                ws[(wave * RB + r) * CAND + j] = bs;
                wi[(wave * RB + r) * CAND + j] = bi;
            }
        });
    }
    __syncthreads();
    if (wave < RB) {
        const int r = wave;
        constexpr int PER = kWaves * CAND / 64;
        TopList<PER> tl;
        tl.init();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = lane + 64 * q;
            const int src = ((e / CAND) * RB + r) * CAND + (e % CAND);
            tl.insert(ws[src], wi[src]);
        }
        const size_t o = (((size_t)grp * RB + r) * n_chunks + chunk) * CAND;
        wave_select<CAND>(tl, [&](int j, float bs, int bi) {
            if (lane == 0) {
                out_s[o + j] = bs;
                out_i[o + j] = bi;
            }
        });
    }
}

// One wave per ROI: the CAND best over its n_lists lists.
template <int CAND>
__global__ __launch_bounds__(256) void k_sparse_merge(const float *__restrict__ in_s, const int32_t *__restrict__ in_i,
                                                      int n_lists, int64_t n_rows, int32_t *__restrict__ cand_idx)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int n = n_lists * CAND;
    const float *s = in_s + (size_t)row * n;
    const int32_t *ix = in_i + (size_t)row * n;
    TopList<CAND> tl;
    tl.init();
    for (int e = lane; e < n; e += 64) tl.insert(s[e], ix[e]);
    wave_select<CAND>(tl, [&](int j, float, int bi) {
        if (lane == 0) cand_idx[(size_t)row * CAND + j] = bi;
    });
}

// One workgroup per ROI: exact FP32 Eq. S1 for each candidate (entries in
// decreasing-value order), then the k best by (Delta, index).
template <int CAND>
__global__ __launch_bounds__(256) void k_sparse_rescore(
    const float *__restrict__ S, const float *__restrict__ inv_s, int n_win, int n_dir,
    const int32_t *__restrict__ strong_idx, const float *__restrict__ strong_val, const uint16_t *__restrict__ lut_gi,
    int n_hat, const int64_t *__restrict__ phase_start, int n_phase, int64_t n_lib,
    const int32_t *__restrict__ cand_idx, int k, int32_t *__restrict__ top_idx, float *__restrict__ top_score)
{
#pragma clang fp contract(off)
    __shared__ float red[256];
    __shared__ float ds[CAND];
    __shared__ int di[CAND];
    const int64_t r = blockIdx.x;
    const float *srow = S + (size_t)r * n_win * n_dir;
    const float *is = inv_s + (size_t)r * n_win;
    for (int c = 0; c < CAND; ++c) {
        const int l = cand_idx[(size_t)r * CAND + c];
        const bool ok = l >= 0 && l < n_lib;
        float acc = 0.0f;
        if (ok) {
            const int ph = phase_of(l, phase_start, n_phase);
            const int32_t *si = strong_idx + (size_t)ph * n_hat;
            const float *sv = strong_val + (size_t)ph * n_hat;
            const uint16_t *row = lut_gi + (size_t)l * n_hat;
            for (int i = threadIdx.x; i < n_hat; i += 256) {
                const int w = si[i] / n_dir;
                const float d = srow[(size_t)w * n_dir + row[i]] * is[w] - sv[i];
                acc = fmaf(d, d, acc);
            }
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            ds[c] = ok ? red[0] : INFINITY;
            di[c] = ok ? l : 0x7fffffff;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int a = 1; a < CAND; ++a) {
            const float vs = ds[a];
            const int vi = di[a];
            int b = a - 1;
            while (b >= 0 && pair_less(vs, vi, ds[b], di[b])) {
                ds[b + 1] = ds[b];
                di[b + 1] = di[b];
                --b;
            }
            ds[b + 1] = vs;
            di[b + 1] = vi;
        }
        for (int j = 0; j < k; ++j) {
            top_idx[(size_t)r * k + j] = di[j] == 0x7fffffff ? -1 : di[j];
            top_score[(size_t)r * k + j] = ds[j];
        }
    }
}

// ROIs per screen workgroup: the largest of 4, 2, 1 whose window slab fits
// the LDS of one workgroup.
int rois_per_block(const ar_context *ctx, int n_dir)
{
    for (int rb = 4; rb > 1; rb >>= 1)
        if ((int64_t)(n_dir * rb + 7) / 8 * 16 <= ctx->lds_per_block) return rb;
    return 1;
}

int64_t slab_halves(int n_dir, int rb) { return ((int64_t)n_dir * rb + 7) / 8 * 8; }

template <int RB, int CAND>
ar_status run_screen(ar_context *ctx, const ar_sparse_lut *lut, const float *images, int64_t n_roi, int k,
                     int32_t *top_idx, float *top_score, hipStream_t s)
{
    const int n_win = lut->n_win, n_dir = lut->n_dir;
    const int64_t n_grp = (n_roi + RB - 1) / RB;
    const int64_t slab = slab_halves(n_dir, RB);
    const size_t lds = std::max((size_t)slab * 2, (size_t)kWaves * RB * CAND * 8);
    AR_CHECK((size_t)ctx->lds_per_block >= lds, "sparse screen needs %zu bytes of LDS", lds);
    AR_CHECK(n_grp < (int64_t)INT32_MAX, "too many ROIs");
    const int64_t n_work = n_grp * lut->n_chunks;
    const int64_t blocks = (n_work + 7) / 8 * 8;
    AR_CHECK(blocks < (int64_t)INT32_MAX, "too many screen workgroups");

    AR_TRY(ctx->sp_half.reserve(sizeof(_Float16) * (size_t)(n_grp * n_win * slab)));
    AR_TRY(ctx->sp_inv.reserve(sizeof(float) * (size_t)(n_roi * n_win)));
    AR_TRY(ctx->sp_cand_s.reserve(sizeof(float) * (size_t)(n_grp * RB * lut->n_chunks * CAND)));
    AR_TRY(ctx->sp_cand_i.reserve(sizeof(int32_t) * (size_t)(n_grp * RB * lut->n_chunks * CAND)));
    AR_TRY(ctx->sp_merge.reserve(sizeof(int32_t) * (size_t)(n_roi * CAND)));

    k_sparse_norm<RB><<<dim3((unsigned)n_grp, (unsigned)n_win), 256, 0, s>>>(
        images, n_roi, n_win, n_dir, slab, ctx->sp_inv.as<float>(), ctx->sp_half.as<_Float16>());
    AR_HIP(hipGetLastError());
    static bool attr_set = false;   // per instantiation
    if (!attr_set && lds > 65536) {
        AR_HIP(hipFuncSetAttribute((const void *)k_sparse_screen<RB, CAND>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    k_sparse_screen<RB, CAND><<<(unsigned)blocks, kThreads, lds, s>>>(
        ctx->sp_half.as<_Float16>(), n_win, slab, lut->lut_ig.as<uint16_t>(), lut->ld, lut->kval2.as<uint32_t>(),
        lut->seg.as<int32_t>(), lut->n_hat, lut->chunks.as<int4>(), lut->n_chunks, (int)n_grp, n_work,
        ctx->sp_cand_s.as<float>(), ctx->sp_cand_i.as<int32_t>());
    AR_HIP(hipGetLastError());
    k_sparse_merge<CAND><<<(unsigned)((n_roi + 3) / 4), 256, 0, s>>>(
        ctx->sp_cand_s.as<float>(), ctx->sp_cand_i.as<int32_t>(), lut->n_chunks, n_roi, ctx->sp_merge.as<int32_t>());
    AR_HIP(hipGetLastError());
    k_sparse_rescore<CAND><<<(unsigned)n_roi, 256, 0, s>>>(
        images, ctx->sp_inv.as<float>(), n_win, n_dir, lut->strong_idx.as<int32_t>(), lut->strong_val.as<float>(),
        lut->lut_gi.as<uint16_t>(), lut->n_hat, lut->phase_start.as<int64_t>(), lut->n_phase, lut->n_lib,
        ctx->sp_merge.as<int32_t>(), k, top_idx, top_score);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // namespace sparse
}  // namespace ar

using namespace ar;

extern "C" {

ar_status ar_sparse_lut_create(ar_context *ctx, const float *reference, int32_t n_phase, int32_t n_win,
                               const float *directions, int32_t n_dir, const double *quats,
                               const int64_t *phase_count, int32_t n_hat, void *stream, ar_sparse_lut **out)
{
    AR_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(reference && directions && quats && phase_count, "NULL argument");
    AR_CHECK(n_phase >= 1 && n_win >= 1, "n_phase and n_win must be >= 1");
    AR_CHECK(n_dir >= 1 && n_dir <= 65535, "n_dir must be in [1, 65535] (16-bit node ids), got %d", n_dir);
    const int64_t K = (int64_t)n_win * n_dir;
    AR_CHECK(n_hat >= 1 && n_hat <= K && n_hat <= 65535, "n_hat must be in [1, min(n_win * n_dir, 65535)], got %d",
             n_hat);
    std::vector<int64_t> start(n_phase + 1, 0);
    for (int c = 0; c < n_phase; ++c) {
        AR_CHECK(phase_count[c] >= 0, "phase_count[%d] < 0", c);
        start[c + 1] = start[c] + phase_count[c];
    }
    const int64_t n_lib = start[n_phase];
    AR_CHECK(n_lib >= 1 && n_lib < (int64_t)INT32_MAX - sparse::kChunk, "library size out of range");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;

    // screen chunks: per phase, columns from the multiple of four at or below its start
    std::vector<int4> ch;
    for (int c = 0; c < n_phase; ++c)
        for (int64_t a = start[c] & ~(int64_t)(sparse::kPerLane - 1); start[c] < start[c + 1] && a < start[c + 1];
             a += sparse::kChunk)
            ch.push_back(make_int4(c, (int)a, (int)std::max(a, start[c]),
                                   (int)std::min(a + sparse::kChunk, start[c + 1])));

    auto *lut = new (std::nothrow) ar_sparse_lut();
    if (!lut) return fail(AR_ENOMEM, "look-up table allocation failed");
    lut->ctx = ctx;
    lut->n_phase = n_phase;
    lut->n_win = n_win;
    lut->n_dir = n_dir;
    lut->n_hat = n_hat;
    lut->n_lib = n_lib;
    lut->ld = (n_lib + sparse::kChunk + 63) / 64 * 64;
    lut->n_chunks = (int32_t)ch.size();
    const size_t nh = (size_t)n_phase * n_hat;
    ar::DeviceBuffer ref_max;
    ar_status st = AR_OK;
    auto step = [&](ar_status x) {
        if (st == AR_OK) st = x;
    };
    auto launched = [&](const char *name) {
        hipError_t e = hipGetLastError();
        if (st == AR_OK && e != hipSuccess) st = fail(AR_EDEVICE, "%s: %s", name, hipGetErrorString(e));
    };
    step(lut->phase_start.reserve(sizeof(int64_t) * (n_phase + 1)));
    step(lut->strong_idx.reserve(sizeof(int32_t) * nh));
    step(lut->strong_val.reserve(sizeof(float) * nh));
    step(lut->kpos.reserve(sizeof(int32_t) * nh));
    step(lut->kval2.reserve(sizeof(uint32_t) * nh));
    step(lut->seg.reserve(sizeof(int32_t) * n_phase * (n_win + 1)));
    step(lut->lut_ig.reserve(sizeof(uint16_t) * (size_t)n_hat * lut->ld));
    step(lut->lut_gi.reserve(sizeof(uint16_t) * (size_t)n_lib * n_hat));
    step(lut->chunks.reserve(sizeof(int4) * ch.size()));
    step(ref_max.reserve(sizeof(float) * n_phase * n_win));
    if (st == AR_OK) {
        hipError_t e = hipMemcpyAsync(lut->phase_start.ptr, start.data(), sizeof(int64_t) * (n_phase + 1),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lut->chunks.ptr, ch.data(), sizeof(int4) * ch.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(lut->lut_ig.ptr, 0, sizeof(uint16_t) * (size_t)n_hat * lut->ld, s);
        if (e != hipSuccess) st = fail(AR_EDEVICE, "look-up table upload: %s", hipGetErrorString(e));
    }
    if (st == AR_OK) {
        sparse::k_ref_max<<<(unsigned)(n_phase * n_win), 256, 0, s>>>(reference, n_dir, ref_max.as<float>());
        launched("k_ref_max");
    }
    if (st == AR_OK) {
        sparse::k_strong_rank<<<dim3((unsigned)((K + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            reference, ref_max.as<float>(), n_win, n_dir, n_hat, lut->strong_idx.as<int32_t>(),
            lut->strong_val.as<float>());
        launched("k_strong_rank");
    }
    if (st == AR_OK) {
        sparse::k_window_order<<<dim3((unsigned)((n_hat + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            lut->strong_idx.as<int32_t>(), lut->strong_val.as<float>(), n_hat, n_win, n_dir, lut->kpos.as<int32_t>(),
            lut->kval2.as<uint32_t>(), lut->seg.as<int32_t>());
        launched("k_window_order");
    }
    if (st == AR_OK) {
        sparse::k_sparse_lut<<<dim3((unsigned)((n_lib + 255) / 256), (unsigned)n_hat), 256, 0, s>>>(
            quats, lut->phase_start.as<int64_t>(), n_phase, n_lib, lut->strong_idx.as<int32_t>(),
            lut->kpos.as<int32_t>(), n_hat, directions, n_dir, lut->lut_ig.as<uint16_t>(), lut->ld);
        launched("k_sparse_lut");
    }
    if (st == AR_OK) {
        const int64_t n = n_lib * n_hat;
        sparse::k_lut_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            lut->lut_ig.as<uint16_t>(), lut->ld, lut->kpos.as<int32_t>(), lut->phase_start.as<int64_t>(), n_phase,
            n_lib, n_hat, lut->lut_gi.as<uint16_t>());
        launched("k_lut_rows");
    }
    // ref_max is freed on return: hipFree waits for the kernels that read it
    if (st != AR_OK) {
        delete lut;
        return st;
    }
    *out = lut;
    return AR_OK;
}

ar_status ar_sparse_lut_destroy(ar_sparse_lut *lut)
{
    if (!lut) return AR_OK;
    (void)hipSetDevice(lut->ctx->device);
    (void)hipDeviceSynchronize();
    delete lut;
    return AR_OK;
}

ar_status ar_sparse_lut_export(const ar_sparse_lut *lut, int32_t *strong_idx, float *strong_val, int32_t *nodes,
                               void *stream)
{
    AR_CHECK(lut != nullptr, "look-up table is NULL");
    AR_HIP(hipSetDevice(lut->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const size_t nh = (size_t)lut->n_phase * lut->n_hat;
    if (strong_idx)
        AR_HIP(hipMemcpyAsync(strong_idx, lut->strong_idx.ptr, sizeof(int32_t) * nh, hipMemcpyDeviceToDevice, s));
    if (strong_val)
        AR_HIP(hipMemcpyAsync(strong_val, lut->strong_val.ptr, sizeof(float) * nh, hipMemcpyDeviceToDevice, s));
    if (nodes) {
        const int64_t n = lut->n_lib * lut->n_hat;
        sparse::k_lut_export<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lut->lut_gi.as<uint16_t>(), n, nodes);
        AR_HIP(hipGetLastError());
    }
    return AR_OK;
}

ar_status index_orientations_sparse(ar_context *ctx, const float *images, int64_t n_roi, const ar_sparse_lut *lut,
                                    int32_t k, int32_t *top_idx, float *top_score, void *stream)
{
    AR_CHECK(ctx && lut, "ctx/look-up table is NULL");
    AR_CHECK(images && top_idx && top_score, "images/top_idx/top_score must not be NULL");
    AR_CHECK(n_roi >= 1 && n_roi < (int64_t)INT32_MAX, "n_roi out of range");
    AR_CHECK(k >= 1 && k <= 32, "k must be in [1, 32], got %d", k);
    AR_CHECK(lut->ctx == ctx, "look-up table belongs to another context");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int rb = sparse::rois_per_block(ctx, lut->n_dir);
    if (k <= 16) {
        if (rb == 4) return sparse::run_screen<4, 16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
        if (rb == 2) return sparse::run_screen<2, 16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
        return sparse::run_screen<1, 16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    }
    if (rb == 4) return sparse::run_screen<4, 32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    if (rb == 2) return sparse::run_screen<2, 32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    return sparse::run_screen<1, 32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
}

}  // extern "C"
