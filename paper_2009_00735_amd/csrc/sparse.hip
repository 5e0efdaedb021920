// Sparse orientation indexing: Eq. S1 evaluated at the strongest reference
// entries through a look-up table of rotated nodes (supplement, "Indexing
// algorithm"; creation cost O_lu = N_c N_g N^_v and indexing cost
// O_idx = N_roi N_c N_g N^_v of the complexity paragraph).
//
// Look-up table (ar_sparse_lut_create), per phase c:
//   1. k_ref_max        per window, the maximum of the raw reference image.
//   2. k_strong_keys    every entry's key x / max in FP64 (+0 for -0); the
//                       n_hat largest keys, equal keys by the lower flat
//                       index w * n_dir + v, in that order: k_strong_threshold
//                       finds the n_hat-th largest key a digit at a time,
//                       k_strong_compact keeps the keys above it and the
//                       lowest-index ties at it, k_strong_place puts each
//                       kept entry at its rank.
//   3. k_window_count   strong entries per window; the host pads every
//                       window's segment to a multiple of 4 rows.
//   4. k_window_order   the strong entries regrouped by window (stable) into
//                       the padded rows the screens walk, with their values as
//                       FP16 pairs and as 8-bit codes round(255 R) (padding
//                       rows: value 0, node = the zero node n_dir).
//   5. k_sparse_lut     for every orientation g of phase c and strong entry i:
//                       the mesh node closest to R(q_g) n_{v_i}.
//   6. k_lut_rows       the same table transposed to one row per orientation,
//                       entries in window order (unpadded), for the rescore.
//
// Indexing (index_orientations_sparse): a screen keeps CAND candidates per
// ROI, k_sparse_merge combines the orientation chunks and k_sparse_rescore
// evaluates exact FP32 Eq. S1 for the candidates from the FP32 image.  Each
// screen workgroup takes (a chunk of 4096 orientations of one phase, a group
// of ROIs): for each window the group's ROI images of that window sit in LDS
// (node-major, plus a zero node), every lane owns four orientations and reads
// their node ids with one 8-byte load per strong entry.  Two screens:
//   * k_sparse_screen8 (meshes whose 8-ROI slab fits LDS): 8 ROIs per node as
//     8-bit codes round(255 s) in one 8-byte LDS read; per lane and
//     orientation, four entries' reads are byte-transposed (v_perm_b32) so
//     that v_dot4_u32_u8 accumulates sum s^2 and sum s R exactly in integers;
//     score = sum s^2 - 2 sum s R + sum R^2 (in 255^2 units).
//   * k_sparse_screen<RB> (wider meshes, RB = 2 or 1): RB ROIs per node in
//     FP16; s - R in packed FP16 (v_pk_add_f16), squares accumulated in FP32
//     (v_fma_mix_f32).
// Either way the workgroup keeps the CAND best orientations per ROI
// (per-wave selection, then a merge in LDS).
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
    int32_t n_rows = 0;                  // screen rows per phase (window segments padded to multiples of 4)
    int32_t n_chunks = 0;
    int32_t screen = 0;                  // 8: 8-bit screen with 8 ROIs per read; 2, 1: FP16 screen with RB ROIs
    ar::DeviceBuffer phase_start;        // int64 [n_phase + 1]
    ar::DeviceBuffer strong_idx;         // int32 [n_phase][n_hat], w * n_dir + v, decreasing value
    ar::DeviceBuffer strong_val;         // float [n_phase][n_hat], normalised value
    ar::DeviceBuffer kpos;               // int32 [n_phase][n_hat], screen row of entry i
    ar::DeviceBuffer kval2;              // uint32 [n_phase][n_rows]: (R, R) in FP16 per screen row
    ar::DeviceBuffer kq8;                // uint8 [n_phase][n_rows]: round(255 R) per screen row
    ar::DeviceBuffer q2sum;              // uint32 [n_phase]: sum of the squared 8-bit codes
    ar::DeviceBuffer seg;                // int32 [n_phase][n_win + 1], padded window segments of the screen rows
    ar::DeviceBuffer lut_ig;             // uint16 [n_rows][ld], screen rows of each column's phase
    ar::DeviceBuffer kcmp;               // int32 [n_phase][n_hat], unpadded window-order position of entry i
    ar::DeviceBuffer cseg;               // int32 [n_phase][n_win + 1], unpadded window segments
    ar::DeviceBuffer sval_w;             // float [n_phase][n_hat], strong values in window order
    ar::DeviceBuffer lut_gi;             // uint16 [n_lib][n_hat], window order (kcmp)
    ar::DeviceBuffer chunks;             // int4 [n_chunks]: phase, first column (multiple of 4), valid [lo, hi)
};

namespace ar {
namespace sparse {

constexpr int kThreads = 1024;               // screen workgroup: 16 waves
constexpr int kWaves = kThreads / 64;
constexpr int kPerLane = 4;                  // orientations per lane (FP16 screens)
constexpr int kPerLane8 = 2;                 // orientations per lane (8-bit screen)
constexpr int kChunk = kPerLane * kThreads;  // largest chunk: orientations per workgroup

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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

// grid (ceil(K / 256), n_phase): key[c][e] = x / max of window e / n_dir in
// FP64 (0 for an all-zero window), -0 made +0 so that equal keys have equal
// codes.
__global__ __launch_bounds__(256) void k_strong_keys(const float *__restrict__ ref, const float *__restrict__ ref_max,
                                                     int n_win, int n_dir, double *__restrict__ key)
{
    const int c = blockIdx.y;
    const int64_t K = (int64_t)n_win * n_dir;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= K) return;
    const float m = ref_max[(size_t)c * n_win + e / n_dir];
    key[(size_t)c * K + e] = (m > 0.0f ? (double)ref[(size_t)c * K + e] / (double)m : 0.0) + 0.0;
}

// Order-preserving code of a double: a larger value has a larger code.
__device__ __forceinline__ uint64_t key_code(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

constexpr int kSelThreads = 1024;

// One workgroup per phase: thr[c] = the n_hat-th largest key code T and
// n_gt[c] = the number of codes above it (fewer than n_hat).  T is found one
// 8-bit digit at a time from the top: a histogram of the digit over the codes
// that match the digits found so far, then the digit at which the count from
// the top reaches the number still to place.
__global__ __launch_bounds__(kSelThreads) void k_strong_threshold(const double *__restrict__ key, int64_t K, int n_hat,
                                                                  uint64_t *__restrict__ thr, int32_t *__restrict__ n_gt)
{
    __shared__ int hist[256];
    __shared__ int pick[2];   // digit, count above it
    const double *k = key + (size_t)blockIdx.x * K;
    uint64_t prefix = 0, mask = 0;
    int need = n_hat;         // codes still to place at or below the prefix
    for (int d = 7; d >= 0; --d) {
        for (int i = threadIdx.x; i < 256; i += kSelThreads) hist[i] = 0;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < K; e += kSelThreads) {
            const uint64_t code = key_code(k[e]);
            if ((code & mask) == prefix) atomicAdd(&hist[(int)((code >> (8 * d)) & 255u)], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int above = 0, b = 255;
            for (; b > 0 && above + hist[b] < need; --b) above += hist[b];
            pick[0] = b;
            pick[1] = above;
        }
        __syncthreads();
        prefix |= (uint64_t)pick[0] << (8 * d);
        mask |= (uint64_t)255u << (8 * d);
        need -= pick[1];
        __syncthreads();   // pick and hist are rewritten by the next digit
    }
    if (threadIdx.x == 0) {
        thr[blockIdx.x] = prefix;
        n_gt[blockIdx.x] = n_hat - need;
    }
}

// One workgroup per phase, entries in index order: keep every code above T
// and the first n_hat - n_gt codes equal to it; the kept entries go, in
// index order, to sel_key / sel_idx [c][0 .. n_hat).
__global__ __launch_bounds__(kSelThreads) void k_strong_compact(const double *__restrict__ key, int64_t K, int n_hat,
                                                                const uint64_t *__restrict__ thr,
                                                                const int32_t *__restrict__ n_gt,
                                                                double *__restrict__ sel_key, int32_t *__restrict__ sel_idx)
{
    __shared__ int wsel[kSelThreads / 64], weq[kSelThreads / 64];
    const int c = blockIdx.x;
    const double *k = key + (size_t)c * K;
    const uint64_t T = thr[c];
    const int ties = n_hat - n_gt[c];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1;
    int eq_base = 0, sel_base = 0;   // ties and kept entries before this chunk
    for (int64_t c0 = 0; c0 < K; c0 += kSelThreads) {
        const int64_t e = c0 + threadIdx.x;
        const double x = e < K ? k[e] : 0.0;
        const uint64_t code = e < K ? key_code(x) : 0;
        const bool eq = e < K && code == T;
        // tie rank in index order: ties in earlier waves of the chunk, then lanes below
        const uint64_t beq = __ballot(eq);
        if (lane == 0) weq[wave] = __popcll(beq);
        __syncthreads();
        int eq_before = eq_base + __popcll(beq & lt), eq_chunk = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) {
            if (w < wave) eq_before += weq[w];
            eq_chunk += weq[w];
        }
        const bool keep = e < K && (code > T || (eq && eq_before < ties));
        const uint64_t bsel = __ballot(keep);
        if (lane == 0) wsel[wave] = __popcll(bsel);
        __syncthreads();
        int pos = sel_base + __popcll(bsel & lt), sel_chunk = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) {
            if (w < wave) pos += wsel[w];
            sel_chunk += wsel[w];
        }
        if (keep) {
            sel_key[(size_t)c * n_hat + pos] = x;
            sel_idx[(size_t)c * n_hat + pos] = (int32_t)e;
        }
        eq_base += eq_chunk;
        sel_base += sel_chunk;
        __syncthreads();   // wsel / weq are rewritten by the next chunk
    }
}

// grid (ceil(n_hat / 256), n_phase): kept entry i goes to its rank among the
// kept ones (larger key first, equal keys by lower index).
__global__ __launch_bounds__(256) void k_strong_place(const double *__restrict__ sel_key,
                                                     const int32_t *__restrict__ sel_idx, int n_hat,
                                                     int32_t *__restrict__ strong_idx, float *__restrict__ strong_val)
{
    const int c = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_hat) return;
    const double *sk = sel_key + (size_t)c * n_hat;
    const int32_t *si = sel_idx + (size_t)c * n_hat;
    const uint64_t ki = key_code(sk[i]);
    const int32_t ii = si[i];
    int rank = 0;
    for (int j = 0; j < n_hat; ++j) {
        const uint64_t kj = key_code(sk[j]);
        rank += kj > ki || (kj == ki && si[j] < ii);
    }
    strong_idx[(size_t)c * n_hat + rank] = ii;
    strong_val[(size_t)c * n_hat + rank] = (float)sk[i];
}

// grid (ceil(n_hat / 256), n_phase): strong entries per window (count is zeroed)
__global__ __launch_bounds__(256) void k_window_count(const int32_t *__restrict__ strong_idx, int n_hat, int n_win,
                                                      int n_dir, int32_t *__restrict__ count)
{
    const int c = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_hat) atomicAdd(&count[(size_t)c * n_win + strong_idx[(size_t)c * n_hat + i] / n_dir], 1);
}

// grid (ceil(n_hat / 256), n_phase): screen row of strong entry i = the
// padded start of its window + its rank among the entries of that window;
// the row's FP16 pair and 8-bit code; q2sum[c] accumulates the squared codes.
__global__ __launch_bounds__(256) void k_window_order(const int32_t *__restrict__ strong_idx,
                                                      const float *__restrict__ strong_val, int n_hat, int n_win,
                                                      int n_dir, const int32_t *__restrict__ seg,
                                                      const int32_t *__restrict__ cseg, int n_rows,
                                                      int32_t *__restrict__ kpos, int32_t *__restrict__ kcmp,
                                                      float *__restrict__ sval_w, uint32_t *__restrict__ kval2,
                                                      uint8_t *__restrict__ kq8, uint32_t *__restrict__ q2sum)
{
    const int c = blockIdx.y;
    const int32_t *si = strong_idx + (size_t)c * n_hat;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_hat) return;
    const int wi = si[i] / n_dir;
    int rank = 0;
    for (int j = 0; j < i; ++j) rank += (si[j] / n_dir == wi) ? 1 : 0;
    const int pos = seg[(size_t)c * (n_win + 1) + wi] + rank;
    const int cpos = cseg[(size_t)c * (n_win + 1) + wi] + rank;
    kpos[(size_t)c * n_hat + i] = pos;
    kcmp[(size_t)c * n_hat + i] = cpos;
    const float v = strong_val[(size_t)c * n_hat + i];
    sval_w[(size_t)c * n_hat + cpos] = v;
    const _Float16 h = (_Float16)v;
    kval2[(size_t)c * n_rows + pos] = __builtin_bit_cast(uint32_t, half2_t{h, h});
    const uint32_t q = (uint32_t)rintf(255.0f * fminf(fmaxf(v, 0.0f), 1.0f));
    kq8[(size_t)c * n_rows + pos] = (uint8_t)q;
    atomicAdd(&q2sum[c], q * q);
}

__global__ __launch_bounds__(256) void k_fill_u16(uint16_t *__restrict__ p, int64_t n, uint16_t v)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) p[t] = v;
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
                                                    const float *__restrict__ dirs, int n_dir, MeshCells mc,
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
    const int p = nearest_node(rx, ry, rz, dirs, n_dir, mc);
    if (valid) lut_ig[(size_t)kpos[(size_t)c * n_hat + i] * ld + g] = (uint16_t)p;
}

// one thread per (orientation, entry in decreasing-value order)
__global__ __launch_bounds__(256) void k_lut_rows(const uint16_t *__restrict__ lut_ig, int64_t ld,
                                                  const int32_t *__restrict__ kpos, const int32_t *__restrict__ kcmp,
                                                  const int64_t *__restrict__ phase_start, int n_phase,
                                                  int64_t n_lib, int n_hat, uint16_t *__restrict__ lut_gi)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_lib * n_hat) return;
    const int64_t g = t / n_hat;
    const int i = (int)(t - g * n_hat);
    const int c = phase_of(g, phase_start, n_phase);
    lut_gi[(size_t)g * n_hat + kcmp[(size_t)c * n_hat + i]] = lut_ig[(size_t)kpos[(size_t)c * n_hat + i] * ld + g];
}

// out[g][i] in decreasing-value order from the window-ordered rows
__global__ __launch_bounds__(256) void k_lut_export(const uint16_t *__restrict__ lut_gi,
                                                    const int32_t *__restrict__ kcmp,
                                                    const int64_t *__restrict__ phase_start, int n_phase,
                                                    int64_t n_lib, int n_hat, int32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_lib * n_hat) return;
    const int64_t g = t / n_hat;
    const int i = (int)(t - g * n_hat);
    const int c = phase_of(g, phase_start, n_phase);
    out[t] = lut_gi[(size_t)g * n_hat + kcmp[(size_t)c * n_hat + i]];
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

// Per (ROI, window) 1 / max in FP32 (0 for an all-zero window) for RB ROIs of
// a group, block-wide; inv_s[r][w] is written for ROIs below n_roi.
template <int RB>
__device__ __forceinline__ void group_inverse_max(const float *__restrict__ img, int64_t n_roi, int n_win, int n_dir,
                                                  int64_t grp, int w, float *red, float *inv,
                                                  float *__restrict__ inv_s)
{
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
}

// grid (n_grp, n_win).  half[grp][w][slab]: node v of ROI grp * RB + j at half
// index v * RB + j, FP16 of the normalised value; node n_dir (the zero node),
// ROIs past n_roi and the slab padding are zero.
template <int RB>
__global__ __launch_bounds__(256) void k_sparse_norm(const float *__restrict__ img, int64_t n_roi, int n_win, int n_dir,
                                                     int64_t slab, float *__restrict__ inv_s,
                                                     _Float16 *__restrict__ half)
{
    __shared__ float red[256];
    __shared__ float inv[RB];
    const int64_t grp = blockIdx.x;
    const int w = blockIdx.y;
    group_inverse_max<RB>(img, n_roi, n_win, n_dir, grp, w, red, inv, inv_s);
    _Float16 *dst = half + ((size_t)grp * n_win + w) * slab;
    for (int64_t t = threadIdx.x; t < slab; t += 256) {
        const int v = (int)(t / RB), j = (int)(t - (int64_t)v * RB);
        const int64_t r = grp * RB + j;
        float x = 0.0f;
        if (v < n_dir && r < n_roi) x = img[((size_t)r * n_win + w) * n_dir + v] * inv[j];
        dst[t] = (_Float16)x;
    }
}

// grid (n_grp, n_win), 8 ROIs per group.  q8[grp][w][slab bytes]: byte
// v * 8 + j = round(255 s) of ROI grp * 8 + j at node v, s the normalised value
// (clamped to [0, 1]); node n_dir, ROIs past n_roi and padding are zero.  The
// eight window maxima are taken together (one pass, eight loads in flight).
__global__ __launch_bounds__(256) void k_sparse_norm8(const float *__restrict__ img, int64_t n_roi, int n_win,
                                                      int n_dir, int64_t slab, float *__restrict__ inv_s,
                                                      uint32_t *__restrict__ q8)
{
    __shared__ float part[4][8];
    __shared__ float inv[8];
    const int64_t grp = blockIdx.x;
    const int w = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nr = (int)min((int64_t)8, n_roi - grp * 8);
    const float *src = img + ((size_t)grp * 8 * n_win + w) * n_dir;   // ROI j at src + j * n_win * n_dir
    const size_t rs = (size_t)n_win * n_dir;
    // a thread takes four nodes (stride 256) of all eight ROIs per step: 32
    // independent loads in flight
    float m[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) m[j] = 0.0f;
    for (int v0 = tid; v0 < n_dir; v0 += 1024)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int v = v0 + 256 * e;
                if (j < nr && v < n_dir) m[j] = fmaxf(m[j], src[j * rs + v]);
            }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m[j] = fmaxf(m[j], __shfl_xor(m[j], off));
        if (lane == 0) part[wave][j] = m[j];
    }
    __syncthreads();
    if (tid < 8) {
        const float mx = fmaxf(fmaxf(part[0][tid], part[1][tid]), fmaxf(part[2][tid], part[3][tid]));
        inv[tid] = mx > 0.0f ? 1.0f / mx : 0.0f;
        if (tid < nr) inv_s[(size_t)(grp * 8 + tid) * n_win + w] = inv[tid];
    }
    __syncthreads();
    float iv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) iv[j] = inv[j];
    // node v's two words (ROIs 0-3, 4-7); four nodes per thread and step
    uint2 *dst = reinterpret_cast<uint2 *>(q8 + ((size_t)grp * n_win + w) * (slab >> 2));
    const int n_nodes = (int)(slab >> 3);   // slab / 8 bytes: nodes incl. the zero node and padding
    for (int v0 = tid; v0 < n_nodes; v0 += 1024) {
        float x[4][8];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int v = v0 + 256 * e;
                x[e][j] = (j < nr && v < n_dir) ? src[j * rs + v] : 0.0f;
            }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int v = v0 + 256 * e;
            if (v >= n_nodes) break;
            uint32_t word[2] = {0u, 0u};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                word[j >> 2] |= (uint32_t)rintf(255.0f * fminf(fmaxf(x[e][j] * iv[j], 0.0f), 1.0f)) << (8 * (j & 3));
            dst[v] = make_uint2(word[0], word[1]);
        }
    }
}

// Bytes (r, r+1, r+2, r+3 of dword a_k) regrouped per r: t[r] byte k = byte r
// of a_k (a 4 x 4 byte transpose, eight v_perm_b32).
__device__ __forceinline__ void transpose4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t (&t)[4])
{
    const uint32_t p0 = __builtin_amdgcn_perm(a1, a0, 0x05010400u);   // a0.0 a1.0 a0.1 a1.1
    const uint32_t p1 = __builtin_amdgcn_perm(a1, a0, 0x07030602u);   // a0.2 a1.2 a0.3 a1.3
    const uint32_t p2 = __builtin_amdgcn_perm(a3, a2, 0x05010400u);   // a2.0 a3.0 a2.1 a3.1
    const uint32_t p3 = __builtin_amdgcn_perm(a3, a2, 0x07030602u);   // a2.2 a3.2 a2.3 a3.3
    t[0] = __builtin_amdgcn_perm(p2, p0, 0x05040100u);
    t[1] = __builtin_amdgcn_perm(p2, p0, 0x07060302u);
    t[2] = __builtin_amdgcn_perm(p3, p1, 0x05040100u);
    t[3] = __builtin_amdgcn_perm(p3, p1, 0x07060302u);
}

// The work item of a screen workgroup: the (chunk, ROI group) items are
// padded to a multiple of 8 workgroups; item t runs on XCD t / (grid / 8), so
// the 32 compute units of an XCD share the look-up rows of one chunk in L2.
__device__ __forceinline__ bool screen_item(int64_t n_work, int n_grp, int &chunk, int &grp)
{
    const int64_t nb8 = gridDim.x >> 3;
    const int64_t t = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (t >= n_work) return false;
    chunk = (int)(t / n_grp);
    grp = (int)(t - (int64_t)chunk * n_grp);
    return true;
}

// Copy `bytes` (a multiple of 16) from global memory to LDS address 0.
__device__ __forceinline__ void fill_slab(const void *src, int64_t bytes)
{
    const u32x4 *s = reinterpret_cast<const u32x4 *>(src);
    const int n16 = (int)(bytes >> 4);
    for (int q = threadIdx.x; q < n16; q += kThreads) *lds_at<u32x4>(16u * q) = s[q];
}

// The CAND best orientations of the chunk per ROI: per-wave selection over
// the lanes' orientations, then one merge wave per ROI over the wave lists in
// LDS.  out_s/out_i: [n_grp * RB][n_chunks][CAND].
template <int PL, int RB, int CAND, typename Score>
__device__ __forceinline__ void screen_topk(const int4 &ch, int chunk, int grp, int n_chunks, Score score,
                                            float *__restrict__ out_s, int32_t *__restrict__ out_i)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    __syncthreads();   // every wave is done with the slab; LDS now holds the wave lists
    float *ws = reinterpret_cast<float *>(smem);
    int32_t *wi = reinterpret_cast<int32_t *>(smem + sizeof(float) * kWaves * RB * CAND);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        TopList<PL> tl;
        tl.init();
#pragma unroll
        for (int g = 0; g < PL; ++g) {
            const int gi = ch.y + PL * tid + g;
            if (gi >= ch.z && gi < ch.w) tl.insert(score(g, r), gi);
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

// FP16 screen, RB ROIs per node.  Window segments are multiples of 4 rows.
template <int RB, int CAND>
__global__ __launch_bounds__(kThreads) void k_sparse_screen(
    const _Float16 *__restrict__ half, int n_win, int64_t slab, const uint16_t *__restrict__ lut_ig, int64_t ld,
    const uint32_t *__restrict__ kval2, const int32_t *__restrict__ seg, int n_rows, const int4 *__restrict__ chunks,
    int n_chunks, int n_grp, int64_t n_work, float *__restrict__ out_s, int32_t *__restrict__ out_i)
{
    int chunk, grp;
    if (!screen_item(n_work, n_grp, chunk, grp)) return;
    const int4 ch = chunks[chunk];
    // each lane owns orientations ch.y + 4 tid .. + 3: one 8-byte load of
    // their four node ids per screen row
    const uint16_t *lut_c = lut_ig + ch.y;
    const unsigned utid = threadIdx.x;
    const uint32_t *kv2 = kval2 + (size_t)ch.x * n_rows;
    const int32_t *sg = seg + (size_t)ch.x * (n_win + 1);

    float acc[kPerLane][RB];
#pragma unroll
    for (int g = 0; g < kPerLane; ++g)
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[g][r] = 0.0f;

    constexpr int SH = RoiVec<RB>::SHIFT;
    for (int w = 0; w < n_win; ++w) {
        const int j0 = sg[w], j1 = sg[w + 1];
        if (j0 == j1) continue;
        __syncthreads();   // every wave is done with the previous window
        fill_slab(half + ((size_t)grp * n_win + w) * slab, slab * 2);
        __syncthreads();
        for (int j = j0; j < j1; j += 4) {
            uint2 pr[4];
            uint32_t R2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pr[u] = reinterpret_cast<const uint2 *>(lut_c + (size_t)(j + u) * ld)[utid];
                R2[u] = kv2[j + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                RoiVec<RB>::acc(node_offset<SH, 0>(pr[u].x), R2[u], acc[0]);
                RoiVec<RB>::acc(node_offset<SH, 1>(pr[u].x), R2[u], acc[1]);
                RoiVec<RB>::acc(node_offset<SH, 0>(pr[u].y), R2[u], acc[2]);
                RoiVec<RB>::acc(node_offset<SH, 1>(pr[u].y), R2[u], acc[3]);
            }
        }
    }
    screen_topk<kPerLane, RB, CAND>(ch, chunk, grp, n_chunks, [&](int g, int r) { return acc[g][r]; }, out_s, out_i);
}

// 8-bit screen, 8 ROIs per node (one 8-byte read); each lane owns two
// orientations (a 4-byte load of their node ids per row).  Per lane and
// orientation, the reads of four rows are byte-transposed so that one
// v_dot4_u32_u8 adds four rows of s^2 (or s R) for one ROI.  Score in 255^2
// units: sum s^2 - 2 sum s R + sum R^2, an exact integer, as FP32.
//
// Software pipeline over groups of four rows: the node ids of group i + 2
// load from global memory and the LDS reads of group i + 1 are in flight
// while group i is scored; the reference codes of the phase sit in LDS
// behind the slab, so every LDS wait is in order.  LDS layout: the slab
// [0, slab), the phase's codes [slab, slab + n_rows); after the last window
// the scores [8][kChunk8] from 0.  Two waves per ROI then take the CAND best
// of 1024 orientations each: out_s/out_i [n_grp * 8][n_chunks][2][CAND].
constexpr int kChunk8 = kPerLane8 * kThreads;

size_t screen8_lds(int64_t slab, int n_rows)
{
    return std::max((size_t)slab + (size_t)(n_rows + 15) / 16 * 16, sizeof(float) * 8 * kChunk8);
}

template <int CAND>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sparse_screen8(
    const uint32_t *__restrict__ q8, int n_win, int64_t slab, const uint16_t *__restrict__ lut_ig, int64_t ld,
    const uint32_t *__restrict__ kq4, const uint32_t *__restrict__ q2sum, const int32_t *__restrict__ seg, int n_rows,
    const int4 *__restrict__ chunks, int n_chunks, int n_grp, int64_t n_work, float *__restrict__ out_s,
    int32_t *__restrict__ out_i)
{
    int chunk, grp;
    if (!screen_item(n_work, n_grp, chunk, grp)) return;
    const int4 ch = chunks[chunk];
    const int tid = threadIdx.x;
    const int32_t *sg = seg + (size_t)ch.x * (n_win + 1);
    const uint32_t rq = (uint32_t)slab;   // LDS byte offset of row 0's code
    {
        const uint32_t *src = kq4 + (size_t)ch.x * (n_rows >> 2);
        for (int q = tid; q < (n_rows >> 2); q += kThreads) *lds_at<uint32_t>(rq + 4u * q) = src[q];
    }

    uint32_t ss[kPerLane8][8], sr[kPerLane8][8];
#pragma unroll
    for (int g = 0; g < kPerLane8; ++g)
#pragma unroll
        for (int r = 0; r < 8; ++r) ss[g][r] = sr[g][r] = 0u;

    struct Rows {
        u32x2 x[kPerLane8][4];   // 8 codes per node, rows j .. j + 3
        uint32_t R4;             // the four rows' reference codes
    };
    const int64_t step = ld >> 1;   // one row of node ids in 4-byte words
    const uint32_t *base = reinterpret_cast<const uint32_t *>(lut_ig + ch.y) + tid;
    auto load4 = [&](uint32_t (&pr)[4], int j) {
        const uint32_t *p = base + (int64_t)j * step;
#pragma unroll
        for (int u = 0; u < 4; ++u) pr[u] = p[u * step];
    };
    auto gather = [&](const uint32_t (&pr)[4], int j, Rows &v) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v.x[0][u] = *lds_at<const u32x2>(node_offset<3, 0>(pr[u]));
            v.x[1][u] = *lds_at<const u32x2>(node_offset<3, 1>(pr[u]));
        }
        v.R4 = *lds_at<const uint32_t>(rq + (uint32_t)j);
    };
    auto score = [&](const Rows &v) {
#pragma unroll
        for (int g = 0; g < kPerLane8; ++g) {
            uint32_t t[4];
            transpose4(v.x[g][0].x, v.x[g][1].x, v.x[g][2].x, v.x[g][3].x, t);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ss[g][r] = __builtin_amdgcn_udot4(t[r], t[r], ss[g][r], false);
                sr[g][r] = __builtin_amdgcn_udot4(t[r], v.R4, sr[g][r], false);
            }
            transpose4(v.x[g][0].y, v.x[g][1].y, v.x[g][2].y, v.x[g][3].y, t);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ss[g][4 + r] = __builtin_amdgcn_udot4(t[r], t[r], ss[g][4 + r], false);
                sr[g][4 + r] = __builtin_amdgcn_udot4(t[r], v.R4, sr[g][4 + r], false);
            }
        }
    };

    for (int w = 0; w < n_win; ++w) {
        const int j0 = sg[w], j1 = sg[w + 1];
        if (j0 == j1) continue;
        __syncthreads();   // every wave is done with the previous window
        fill_slab(q8 + ((size_t)grp * n_win + w) * (slab >> 2), slab);
        __syncthreads();
        uint32_t pa[4], pb[4];
        Rows va, vb;
        int j = j0;
        if (((j1 - j0) >> 2) & 1) {   // an odd leading group, unpipelined
            load4(pa, j);
            gather(pa, j, va);
            score(va);
            j += 4;
        }
        if (j < j1) {
            // an even number of groups from j: the prefetches past the end
            // repeat the final group and are not scored
            const int last = j1 - 4;
            load4(pa, j);
            load4(pb, j + 4);
            gather(pa, j, va);
            for (; j < j1; j += 8) {
                load4(pa, min(j + 8, last));
                gather(pb, j + 4, vb);
                __builtin_amdgcn_sched_barrier(0);
                score(va);
                __builtin_amdgcn_sched_barrier(0);
                load4(pb, min(j + 12, last));
                gather(pa, min(j + 8, last), va);
                __builtin_amdgcn_sched_barrier(0);
                score(vb);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // scores to LDS, then one merge wave per ROI
    __syncthreads();
    const int64_t c2 = (int64_t)q2sum[ch.x];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int g = 0; g < kPerLane8; ++g)
            *lds_at<float>(4u * (uint32_t)(r * kChunk8 + kPerLane8 * tid + g)) =
                (float)((int64_t)ss[g][r] - 2 * (int64_t)sr[g][r] + c2);
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int r = wave >> 1, half = wave & 1;   // two waves per ROI, 1024 orientations each
    constexpr int PER = kChunk8 / 128;
    TopList<PER> tl;
    tl.init();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = half * (kChunk8 / 2) + lane + 64 * q;
        const int gi = ch.y + e;
        if (gi >= ch.z && gi < ch.w) tl.insert(*lds_at<const float>(4u * (uint32_t)(r * kChunk8 + e)), gi);
    }
    const size_t o = ((((size_t)grp * 8 + r) * n_chunks + chunk) * 2 + half) * CAND;
    wave_select<CAND>(tl, [&](int jj, float bs, int bi) {
        if (lane == 0) {
            out_s[o + jj] = bs;
            out_i[o + jj] = bi;
        }
    });
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

// One workgroup per ROI: exact FP32 Eq. S1 for each candidate, one wave per
// candidate, then the k best by (Delta, index).  The entries of a candidate's
// row come in window order (cseg segments); lane l sums entries l, l + 64, ...
// of each window, windows in order, then a butterfly over the lanes.  STAGE:
// each window of the ROI, normalised in FP32, is first staged in LDS
// (n_dir floats), so the per-entry gathers read LDS; otherwise they read the
// image in global memory.  Either way d = x * (1 / max) - R_i as in the
// screens' normalisation, the square accumulated with one FMA.
template <int CAND, bool STAGE>
__global__ __launch_bounds__(256) void k_sparse_rescore(
    const float *__restrict__ S, const float *__restrict__ inv_s, int n_win, int n_dir,
    const int32_t *__restrict__ cseg, const float *__restrict__ sval_w, const uint16_t *__restrict__ lut_gi,
    int n_hat, const int64_t *__restrict__ phase_start, int n_phase, int64_t n_lib,
    const int32_t *__restrict__ cand_idx, int k, int32_t *__restrict__ top_idx, float *__restrict__ top_score)
{
#pragma clang fp contract(off)
    extern __shared__ float stage[];
    __shared__ float ds[CAND];
    __shared__ int di[CAND];
    constexpr int PER = CAND / 4;   // candidates per wave
    const int64_t r = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float *srow = S + (size_t)r * n_win * n_dir;
    const float *is = inv_s + (size_t)r * n_win;
    int cl[PER], cph[PER];
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int l = cand_idx[(size_t)r * CAND + wave + 4 * q];
        cl[q] = l;
        cph[q] = (l >= 0 && l < n_lib) ? phase_of(l, phase_start, n_phase) : -1;
        acc[q] = 0.0f;
    }
    for (int w = 0; w < n_win; ++w) {
        const float iw = is[w];
        const float *src = srow + (size_t)w * n_dir;
        if (STAGE) {
            __syncthreads();
            // sixteen loads in flight per thread
            for (int v0 = threadIdx.x; v0 < n_dir; v0 += 256 * 16) {
                float x[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) x[e] = v0 + 256 * e < n_dir ? src[v0 + 256 * e] : 0.0f;
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (v0 + 256 * e < n_dir) stage[v0 + 256 * e] = x[e] * iw;
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (cph[q] < 0) continue;
            const int32_t *sg = cseg + (size_t)cph[q] * (n_win + 1);
            const float *sv = sval_w + (size_t)cph[q] * n_hat;
            const uint16_t *row = lut_gi + (size_t)cl[q] * n_hat;
            const int j1 = sg[w + 1];
#pragma unroll 4
            for (int j = sg[w] + lane; j < j1; j += 64) {
                const float x = STAGE ? stage[row[j]] : src[row[j]] * iw;
                const float d = x - sv[j];
                acc[q] = fmaf(d, d, acc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        float a = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (lane == 0) {
            const bool ok = cph[q] >= 0;
            ds[wave + 4 * q] = ok ? a : INFINITY;
            di[wave + 4 * q] = ok ? cl[q] : 0x7fffffff;
        }
    }
    __syncthreads();
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

// Slab bytes of one (ROI group, window): n_dir + 1 nodes (the last is the
// zero node of the padding rows) of `per_node` bytes, rounded up to 16.
int64_t slab_bytes(int n_dir, int per_node) { return ((int64_t)(n_dir + 1) * per_node + 15) / 16 * 16; }

// The screen for a mesh: 8 (8-bit codes, 8 ROIs per node) if that slab and
// n_rows reference codes fit the LDS of one workgroup, else 2 or 1 FP16 ROIs
// per node; 0 if none fits.
int pick_screen(const ar_context *ctx, int n_dir, int n_rows)
{
    if ((int64_t)screen8_lds(slab_bytes(n_dir, 8), n_rows) <= ctx->lds_per_block) return 8;
    if (slab_bytes(n_dir, 4) <= ctx->lds_per_block) return 2;
    if (slab_bytes(n_dir, 2) <= ctx->lds_per_block) return 1;
    return 0;
}

// Dynamic LDS beyond 64 KB must be allowed per kernel; set on every launch
// (on the calling context's device, current at this point).
template <typename K>
ar_status allow_lds(K kernel, size_t lds)
{
    if (lds > 65536) AR_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return AR_OK;
}

// Shared tail of both screens: merge the n_lists lists of each ROI, rescore
// the candidates.
template <int CAND>
ar_status merge_rescore(ar_context *ctx, const ar_sparse_lut *lut, const float *images, int64_t n_roi, int n_lists,
                        int k, int32_t *top_idx, float *top_score, hipStream_t s)
{
    k_sparse_merge<CAND><<<(unsigned)((n_roi + 3) / 4), 256, 0, s>>>(
        ctx->sp_cand_s.as<float>(), ctx->sp_cand_i.as<int32_t>(), n_lists, n_roi, ctx->sp_merge.as<int32_t>());
    AR_HIP(hipGetLastError());
    // stage each ROI window in LDS when n_dir floats fit beside the static arrays
    const size_t stage = sizeof(float) * (size_t)lut->n_dir;
    if (stage + 4096 <= (size_t)ctx->lds_per_block) {
        AR_TRY(allow_lds(k_sparse_rescore<CAND, true>, stage));
        k_sparse_rescore<CAND, true><<<(unsigned)n_roi, 256, stage, s>>>(
            images, ctx->sp_inv.as<float>(), lut->n_win, lut->n_dir, lut->cseg.as<int32_t>(),
            lut->sval_w.as<float>(), lut->lut_gi.as<uint16_t>(), lut->n_hat, lut->phase_start.as<int64_t>(),
            lut->n_phase, lut->n_lib, ctx->sp_merge.as<int32_t>(), k, top_idx, top_score);
    } else {
        k_sparse_rescore<CAND, false><<<(unsigned)n_roi, 256, 0, s>>>(
            images, ctx->sp_inv.as<float>(), lut->n_win, lut->n_dir, lut->cseg.as<int32_t>(),
            lut->sval_w.as<float>(), lut->lut_gi.as<uint16_t>(), lut->n_hat, lut->phase_start.as<int64_t>(),
            lut->n_phase, lut->n_lib, ctx->sp_merge.as<int32_t>(), k, top_idx, top_score);
    }
    AR_HIP(hipGetLastError());
    return AR_OK;
}

// RB ROIs per group (8 for the 8-bit screen): workspace and launch shape.
struct ScreenPlan {
    int64_t n_grp, slab, n_work, blocks;
    size_t lds;
};

template <int RB, int CAND>
ar_status plan_screen(ar_context *ctx, const ar_sparse_lut *lut, int64_t n_roi, int per_node, ScreenPlan &p)
{
    p.n_grp = (n_roi + RB - 1) / RB;
    p.slab = slab_bytes(lut->n_dir, per_node);
    p.lds = std::max((size_t)p.slab, (size_t)kWaves * RB * CAND * 8);
    AR_CHECK((size_t)ctx->lds_per_block >= p.lds, "sparse screen needs %zu bytes of LDS", p.lds);
    AR_CHECK(p.n_grp < (int64_t)INT32_MAX, "too many ROIs");
    p.n_work = p.n_grp * lut->n_chunks;
    p.blocks = (p.n_work + 7) / 8 * 8;
    AR_CHECK(p.blocks < (int64_t)INT32_MAX, "too many screen workgroups");
    AR_TRY(ctx->sp_half.reserve((size_t)(p.n_grp * lut->n_win * p.slab)));
    AR_TRY(ctx->sp_inv.reserve(sizeof(float) * (size_t)(n_roi * lut->n_win)));
    AR_TRY(ctx->sp_cand_s.reserve(sizeof(float) * (size_t)(p.n_grp * RB * lut->n_chunks * CAND)));
    AR_TRY(ctx->sp_cand_i.reserve(sizeof(int32_t) * (size_t)(p.n_grp * RB * lut->n_chunks * CAND)));
    AR_TRY(ctx->sp_merge.reserve(sizeof(int32_t) * (size_t)(n_roi * CAND)));
    return AR_OK;
}


template <int RB, int CAND>
ar_status run_screen(ar_context *ctx, const ar_sparse_lut *lut, const float *images, int64_t n_roi, int k,
                     int32_t *top_idx, float *top_score, hipStream_t s)
{
    ScreenPlan p;
    AR_TRY((plan_screen<RB, CAND>(ctx, lut, n_roi, 2 * RB, p)));
    k_sparse_norm<RB><<<dim3((unsigned)p.n_grp, (unsigned)lut->n_win), 256, 0, s>>>(
        images, n_roi, lut->n_win, lut->n_dir, p.slab / 2, ctx->sp_inv.as<float>(), ctx->sp_half.as<_Float16>());
    AR_HIP(hipGetLastError());
    AR_TRY(allow_lds(k_sparse_screen<RB, CAND>, p.lds));
    k_sparse_screen<RB, CAND><<<(unsigned)p.blocks, kThreads, p.lds, s>>>(
        ctx->sp_half.as<_Float16>(), lut->n_win, p.slab / 2, lut->lut_ig.as<uint16_t>(), lut->ld,
        lut->kval2.as<uint32_t>(), lut->seg.as<int32_t>(), lut->n_rows, lut->chunks.as<int4>(), lut->n_chunks,
        (int)p.n_grp, p.n_work, ctx->sp_cand_s.as<float>(), ctx->sp_cand_i.as<int32_t>());
    AR_HIP(hipGetLastError());
    return merge_rescore<CAND>(ctx, lut, images, n_roi, lut->n_chunks, k, top_idx, top_score, s);
}

template <int CAND>
ar_status run_screen8(ar_context *ctx, const ar_sparse_lut *lut, const float *images, int64_t n_roi, int k,
                      int32_t *top_idx, float *top_score, hipStream_t s)
{
    ScreenPlan p;
    AR_TRY((plan_screen<8, CAND>(ctx, lut, n_roi, 8, p)));
    p.lds = screen8_lds(p.slab, lut->n_rows);
    AR_CHECK((size_t)ctx->lds_per_block >= p.lds, "sparse screen needs %zu bytes of LDS", p.lds);
    AR_TRY(ctx->sp_cand_s.reserve(sizeof(float) * (size_t)(p.n_grp * 8 * lut->n_chunks * 2 * CAND)));
    AR_TRY(ctx->sp_cand_i.reserve(sizeof(int32_t) * (size_t)(p.n_grp * 8 * lut->n_chunks * 2 * CAND)));
    k_sparse_norm8<<<dim3((unsigned)p.n_grp, (unsigned)lut->n_win), 256, 0, s>>>(
        images, n_roi, lut->n_win, lut->n_dir, p.slab, ctx->sp_inv.as<float>(), ctx->sp_half.as<uint32_t>());
    AR_HIP(hipGetLastError());
    AR_TRY(allow_lds(k_sparse_screen8<CAND>, p.lds));
    k_sparse_screen8<CAND><<<(unsigned)p.blocks, kThreads, p.lds, s>>>(
        ctx->sp_half.as<uint32_t>(), lut->n_win, p.slab, lut->lut_ig.as<uint16_t>(), lut->ld,
        lut->kq8.as<uint32_t>(), lut->q2sum.as<uint32_t>(), lut->seg.as<int32_t>(), lut->n_rows,
        lut->chunks.as<int4>(), lut->n_chunks, (int)p.n_grp, p.n_work, ctx->sp_cand_s.as<float>(),
        ctx->sp_cand_i.as<int32_t>());
    AR_HIP(hipGetLastError());
    return merge_rescore<CAND>(ctx, lut, images, n_roi, 2 * lut->n_chunks, k, top_idx, top_score, s);
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
    AR_CHECK(K < (int64_t)INT32_MAX, "n_win * n_dir must be below 2^31");
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

    // screen chunks: per phase, columns from the multiple of four at or below
    // its start, as many per chunk as the screen's workgroup covers
    const int screen = sparse::pick_screen(ctx, n_dir, n_hat + 3 * n_win);   // bound on the padded rows
    const int64_t chunk = (screen == 8 ? sparse::kPerLane8 : sparse::kPerLane) * sparse::kThreads;
    std::vector<int4> ch;
    for (int c = 0; c < n_phase; ++c)
        for (int64_t a = start[c] & ~(int64_t)3; start[c] < start[c + 1] && a < start[c + 1]; a += chunk)
            ch.push_back(make_int4(c, (int)a, (int)std::max(a, start[c]), (int)std::min(a + chunk, start[c + 1])));

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
    lut->screen = screen;
    const size_t nh = (size_t)n_phase * n_hat;
    ar::DeviceBuffer ref_max, count;
    ar_status st = lut->screen ? AR_OK : fail(AR_EINVAL, "no screen layout fits %d nodes in LDS", n_dir);
    auto step = [&](ar_status x) {
        if (st == AR_OK) st = x;
    };
    auto launched = [&](const char *name) {
        hipError_t e = hipGetLastError();
        if (st == AR_OK && e != hipSuccess) st = fail(AR_EDEVICE, "%s: %s", name, hipGetErrorString(e));
    };
    auto hip = [&](hipError_t e, const char *what) {
        if (st == AR_OK && e != hipSuccess) st = fail(AR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    step(lut->phase_start.reserve(sizeof(int64_t) * (n_phase + 1)));
    step(lut->strong_idx.reserve(sizeof(int32_t) * nh));
    step(lut->strong_val.reserve(sizeof(float) * nh));
    step(lut->kpos.reserve(sizeof(int32_t) * nh));
    step(lut->kcmp.reserve(sizeof(int32_t) * nh));
    step(lut->sval_w.reserve(sizeof(float) * nh));
    step(lut->cseg.reserve(sizeof(int32_t) * n_phase * (n_win + 1)));
    step(lut->seg.reserve(sizeof(int32_t) * n_phase * (n_win + 1)));
    step(lut->lut_gi.reserve(sizeof(uint16_t) * (size_t)n_lib * n_hat));
    step(lut->chunks.reserve(sizeof(int4) * ch.size()));
    step(ref_max.reserve(sizeof(float) * n_phase * n_win));
    step(count.reserve(sizeof(int32_t) * n_phase * n_win));
    if (st == AR_OK) {
        hip(hipMemcpyAsync(lut->phase_start.ptr, start.data(), sizeof(int64_t) * (n_phase + 1), hipMemcpyHostToDevice,
                           s), "look-up table upload");
        hip(hipMemcpyAsync(lut->chunks.ptr, ch.data(), sizeof(int4) * ch.size(), hipMemcpyHostToDevice, s),
            "look-up table upload");
        hip(hipMemsetAsync(count.ptr, 0, sizeof(int32_t) * n_phase * n_win, s), "look-up table upload");
    }
    if (st == AR_OK) {
        sparse::k_ref_max<<<(unsigned)(n_phase * n_win), 256, 0, s>>>(reference, n_dir, ref_max.as<float>());
        launched("k_ref_max");
    }
    // strong lists: keys, then the n_hat largest (ties by lower index) in order
    ar::DeviceBuffer keys, sel_key, sel_idx, thr, n_gt;
    step(keys.reserve(sizeof(double) * (size_t)n_phase * K));
    step(sel_key.reserve(sizeof(double) * nh));
    step(sel_idx.reserve(sizeof(int32_t) * nh));
    step(thr.reserve(sizeof(uint64_t) * n_phase));
    step(n_gt.reserve(sizeof(int32_t) * n_phase));
    if (st == AR_OK) {
        sparse::k_strong_keys<<<dim3((unsigned)((K + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            reference, ref_max.as<float>(), n_win, n_dir, keys.as<double>());
        launched("k_strong_keys");
    }
    if (st == AR_OK) {
        sparse::k_strong_threshold<<<(unsigned)n_phase, sparse::kSelThreads, 0, s>>>(
            keys.as<double>(), K, n_hat, thr.as<uint64_t>(), n_gt.as<int32_t>());
        launched("k_strong_threshold");
    }
    if (st == AR_OK) {
        sparse::k_strong_compact<<<(unsigned)n_phase, sparse::kSelThreads, 0, s>>>(
            keys.as<double>(), K, n_hat, thr.as<uint64_t>(), n_gt.as<int32_t>(), sel_key.as<double>(),
            sel_idx.as<int32_t>());
        launched("k_strong_compact");
    }
    if (st == AR_OK) {
        sparse::k_strong_place<<<dim3((unsigned)((n_hat + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            sel_key.as<double>(), sel_idx.as<int32_t>(), n_hat, lut->strong_idx.as<int32_t>(),
            lut->strong_val.as<float>());
        launched("k_strong_place");
    }
    if (st == AR_OK) {
        sparse::k_window_count<<<dim3((unsigned)((n_hat + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            lut->strong_idx.as<int32_t>(), n_hat, n_win, n_dir, count.as<int32_t>());
        launched("k_window_count");
    }
    // padded window segments: every window starts on a multiple of 4 rows
    std::vector<int32_t> cnt((size_t)n_phase * n_win, 0), seg((size_t)n_phase * (n_win + 1), 0),
        cseg((size_t)n_phase * (n_win + 1), 0);
    if (st == AR_OK) {
        hip(hipMemcpyAsync(cnt.data(), count.ptr, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, s),
            "window counts");
        hip(hipStreamSynchronize(s), "window counts");
    }
    int32_t n_rows = 4;
    for (int c = 0; c < n_phase; ++c) {
        int32_t *sc = seg.data() + (size_t)c * (n_win + 1), *cc = cseg.data() + (size_t)c * (n_win + 1);
        for (int w = 0; w < n_win; ++w) {
            sc[w + 1] = sc[w] + (cnt[(size_t)c * n_win + w] + 3) / 4 * 4;
            cc[w + 1] = cc[w] + cnt[(size_t)c * n_win + w];
        }
        n_rows = std::max(n_rows, sc[n_win]);
    }
    lut->n_rows = n_rows;
    const size_t nr = (size_t)n_phase * n_rows;
    step(lut->kval2.reserve(sizeof(uint32_t) * nr));
    step(lut->kq8.reserve(nr));
    step(lut->q2sum.reserve(sizeof(uint32_t) * n_phase));
    step(lut->lut_ig.reserve(sizeof(uint16_t) * (size_t)n_rows * lut->ld));
    if (st == AR_OK) {
        hip(hipMemcpyAsync(lut->seg.ptr, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice, s),
            "look-up table upload");
        hip(hipMemcpyAsync(lut->cseg.ptr, cseg.data(), sizeof(int32_t) * cseg.size(), hipMemcpyHostToDevice, s),
            "look-up table upload");
        hip(hipMemsetAsync(lut->kval2.ptr, 0, sizeof(uint32_t) * nr, s), "look-up table upload");
        hip(hipMemsetAsync(lut->kq8.ptr, 0, nr, s), "look-up table upload");
        hip(hipMemsetAsync(lut->q2sum.ptr, 0, sizeof(uint32_t) * n_phase, s), "look-up table upload");
    }
    if (st == AR_OK) {
        const int64_t n = (int64_t)n_rows * lut->ld;   // padding rows and columns: the zero node
        sparse::k_fill_u16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lut->lut_ig.as<uint16_t>(), n,
                                                                       (uint16_t)n_dir);
        launched("k_fill_u16");
    }
    if (st == AR_OK) {
        sparse::k_window_order<<<dim3((unsigned)((n_hat + 255) / 256), (unsigned)n_phase), 256, 0, s>>>(
            lut->strong_idx.as<int32_t>(), lut->strong_val.as<float>(), n_hat, n_win, n_dir, lut->seg.as<int32_t>(),
            lut->cseg.as<int32_t>(), n_rows, lut->kpos.as<int32_t>(), lut->kcmp.as<int32_t>(),
            lut->sval_w.as<float>(), lut->kval2.as<uint32_t>(), lut->kq8.as<uint8_t>(), lut->q2sum.as<uint32_t>());
        launched("k_window_order");
    }
    MeshCells mc;
    if (st == AR_OK) step(build_mesh_cells(ctx, directions, n_dir, s, mc));
    if (st == AR_OK) {
        sparse::k_sparse_lut<<<dim3((unsigned)((n_lib + 255) / 256), (unsigned)n_hat), 256, 0, s>>>(
            quats, lut->phase_start.as<int64_t>(), n_phase, n_lib, lut->strong_idx.as<int32_t>(),
            lut->kpos.as<int32_t>(), n_hat, directions, n_dir, mc, lut->lut_ig.as<uint16_t>(), lut->ld);
        launched("k_sparse_lut");
    }
    if (st == AR_OK) {
        const int64_t n = n_lib * n_hat;
        sparse::k_lut_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            lut->lut_ig.as<uint16_t>(), lut->ld, lut->kpos.as<int32_t>(), lut->kcmp.as<int32_t>(),
            lut->phase_start.as<int64_t>(), n_phase, n_lib, n_hat, lut->lut_gi.as<uint16_t>());
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
        sparse::k_lut_export<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            lut->lut_gi.as<uint16_t>(), lut->kcmp.as<int32_t>(), lut->phase_start.as<int64_t>(), lut->n_phase,
            lut->n_lib, lut->n_hat, nodes);
        AR_HIP(hipGetLastError());
    }
    return AR_OK;
}

ar_status ar_sparse_lut_screen(const ar_sparse_lut *lut, int32_t *rois_per_read)
{
    AR_CHECK(lut != nullptr && rois_per_read != nullptr, "look-up table or rois_per_read is NULL");
    *rois_per_read = lut->screen;
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
    const int sc = lut->screen;
    if (k <= 16) {
        if (sc == 8) return sparse::run_screen8<16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
        if (sc == 2) return sparse::run_screen<2, 16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
        return sparse::run_screen<1, 16>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    }
    if (sc == 8) return sparse::run_screen8<32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    if (sc == 2) return sparse::run_screen<2, 32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
    return sparse::run_screen<1, 32>(ctx, lut, images, n_roi, k, top_idx, top_score, s);
}

}  // extern "C"
