// Orientation indexing (Sec. 2.4; supplement, "Indexing algorithm",
// Eq. S1): normalised ROI signatures against normalised rotated references
// by the sum of squared differences, read densely over all nodes,
//   Delta(r,l) = |S_r|^2 + |L_l|^2 - 2 <S_r, L_l>.
//
// gfx950 design:
//   1. k_normalise_cast   per (row, window) max over the directions, FP32
//                         reciprocal, BF16 (round to nearest even) copy of the
//                         normalised row, K padded with zeros.
//   2. k_corr_topk        BF16-input / FP32-accumulate MFMA correlation
//                         (v_mfma_f32_32x32x16_bf16), 128x128 workgroup tile,
//                         K in steps of 64 through double-buffered, padded LDS.
//                         Each workgroup owns a 128-row panel and a segment of
//                         library columns; the epilogue turns every tile into
//                         scores |L|^2 - 2<S,L> (the per-row constant |S|^2 is
//                         dropped) and keeps, per row, the CAND best
//                         (score, index) pairs in registers: the ranking
//                         never materialises the score matrix.
//   3. k_merge            per row, the CAND best over all segments.
//   4. k_rescore          exact FP32 sum of squared differences of the
//                         normalised FP32 images for the CAND candidates,
//                         sorted by (Delta, index); the first k are returned.
//                         One workgroup per ROI and one wave per candidate;
//                         each normalised ROI window is staged in LDS once.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ar_internal.h"
#include "topk_device.h"

namespace ar {
namespace idx {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kPadM = 256, kPadN = 256, kPadK = 64;   // multiples of every tile's BM, BN and K step

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------ normalise + cast
// grid (n_rows, n_win); writes inv_max[row][w] and out[row][w*n_dir + v].
// The workgroup of the last window also zeroes the K padding of its row.
__global__ __launch_bounds__(256) void k_normalise_cast(const float *__restrict__ img, int n_win, int n_dir,
                                                        int64_t Kp, float *__restrict__ inv_max,
                                                        uint16_t *__restrict__ out)
{
    __shared__ float red[256];
    const int64_t row = blockIdx.x;
    const int w = blockIdx.y;
    const float *src = img + ((size_t)row * n_win + w) * n_dir;
    float m = 0.0f;
    for (int v = threadIdx.x; v < n_dir; v += blockDim.x) m = fmaxf(m, src[v]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float mx = red[0];
    const float inv = mx > 0.0f ? 1.0f / mx : 0.0f;
    if (threadIdx.x == 0) inv_max[(size_t)row * n_win + w] = inv;
    uint16_t *dst = out + (size_t)row * Kp + (size_t)w * n_dir;
    if ((n_dir & 1) == 0 && (reinterpret_cast<uintptr_t>(img) & 7) == 0) {
        // even n_dir (every geodesic mesh: 10 * 4^k + 2 nodes) and an 8-byte
        // aligned image array: the window's source floats and destination bf16
        // start 8- and 4-byte aligned,
        // so convert pairs with one 8-byte load and one 4-byte store per lane
        const float2 *s2 = reinterpret_cast<const float2 *>(src);
        uint32_t *d2 = reinterpret_cast<uint32_t *>(dst);
        for (int v = threadIdx.x; v < n_dir / 2; v += blockDim.x) {
            const float2 x = s2[v];
            d2[v] = (uint32_t)f32_to_bf16_rne(x.x * inv) | ((uint32_t)f32_to_bf16_rne(x.y * inv) << 16);
        }
    } else {
        for (int v = threadIdx.x; v < n_dir; v += blockDim.x) dst[v] = f32_to_bf16_rne(src[v] * inv);
    }
    if (w == n_win - 1) {
        const int64_t K = (int64_t)n_win * n_dir;
        for (int64_t c = K + threadIdx.x; c < Kp; c += blockDim.x) out[(size_t)row * Kp + c] = 0;
    }
}

// zero rows [r0, r1) of a [*][Kp] bf16 matrix
__global__ __launch_bounds__(256) void k_zero_rows(uint16_t *__restrict__ out, int64_t Kp, int64_t r0, int64_t r1)
{
    const int64_t n = (r1 - r0) * Kp;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[r0 * Kp + i] = 0;
}

// |row|^2 of the BF16 copy, FP32; rows >= n_valid get +inf
__global__ __launch_bounds__(256) void k_row_norm2(const uint16_t *__restrict__ m, int64_t Kp, int64_t n_valid,
                                                   float *__restrict__ norm2)
{
    __shared__ float red[256];
    const int64_t row = blockIdx.x;
    float acc = 0.0f;
    if (row < n_valid)
        for (int64_t c = threadIdx.x; c < Kp; c += blockDim.x) {
            const float x = bf16_to_f32(m[(size_t)row * Kp + c]);
            acc = fmaf(x, x, acc);
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm2[row] = row < n_valid ? red[0] : INFINITY;
}

// ------------------------------------------------------------ correlation
// Workgroup: WGM x WGN waves (2x2 or 2x4); each wave owns WTM x WTN MFMA
// tiles of 32x32 (v_mfma_f32_32x32x16_bf16), so the workgroup tile is
// BM x BN = (32 WTM WGM) x (32 WTN WGN).  K advances 32 bf16 per step.
//
// Operands go straight from global memory into LDS (global_load_lds_dwordx4:
// each wave instruction fills 1 KB = 16 rows of 64 bytes, no registers on the
// way) through a ring of NSTAGE stages, NSTAGE - 1 steps in flight.  Rows are
// unpadded; the 16-byte chunk c of row r sits at chunk c ^ ((r >> 2) & 3),
// which makes the fragment reads (32 consecutive rows, one chunk) free of
// bank conflicts.  One workgroup barrier per step: after it every wave's
// loads of the step have landed and every wave has finished the previous
// step, whose stage is then refilled.
// grid.x = m_blocks * n_seg; the launch covers library rows from col0.
// out_s/out_i: [M_pad][list_stride][CAND]; this launch writes lists
// list_base .. list_base + n_seg * LPR - 1 of each row: with CAND 16 or 32,
// LPR = TPR = THREADS / BM threads share a row in the epilogue, each with its
// own list in registers; with CAND = 64 each wave owns RPW = BM / WAVES whole
// rows, one wave-wide list per row and segment (LPR = 1).
constexpr int kBK = 32;        // bf16 per K step
constexpr int kStages = 4;     // LDS ring depth (5, the most that fits 160 KB at 256 x 256, measured no faster)

template <int WGM, int WGN, int WTM, int WTN> struct CorrShape {
    static constexpr int THREADS = 64 * WGM * WGN, WAVES = WGM * WGN;
    static constexpr int BM = 32 * WTM * WGM, BN = 32 * WTN * WGN;
    static constexpr int ROWB = kBK * 2;                       // bytes per LDS row
    static constexpr int A_BYTES = BM * ROWB, STAGE = (BM + BN) * ROWB;
    static constexpr int A_BLK = BM / 16, B_BLK = BN / 16;     // 1-KB blocks per stage
    static constexpr int BLK_PER_WAVE = (A_BLK + B_BLK) / WAVES;
    static constexpr int TPR = THREADS / BM;                   // epilogue threads per row
    static constexpr int RPW = BM / WAVES;                     // rows per wave (64-entry wave lists)
    static_assert((A_BLK + B_BLK) % WAVES == 0, "stage blocks must split evenly over the waves");
    static constexpr size_t lds()
    {
        const size_t ab = (size_t)kStages * STAGE;
        const size_t c = (size_t)BM * 65 * sizeof(float);
        return ab > c ? ab : c;
    }
};

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt vmcnt(N): this wave's vector-memory operations (here the LDS
// fills) beyond the newest N have completed.
template <int N> __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Instruction order of one K step after its fragment reads: the NF fill
// instructions spread evenly between the NM MFMAs (a run of MFMAs, then one
// fill, NF times).  A wave whose fills all sit in one run stalls at their
// issue while its SIMD's matrix core runs dry; spread out, each fill issues
// behind MFMAs already queued.
template <int I, int NF, int NM> __device__ __forceinline__ void fill_schedule()
{
    if constexpr (I < NF) {
        constexpr int m = NM * (I + 1) / NF - NM * I / NF;
        if constexpr (m > 0) __builtin_amdgcn_sched_group_barrier(0x008, m, 0);   // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                          // VMEM read
        fill_schedule<I + 1, NF, NM>();
    }
}

// Workgroup barrier without a memory fence (a fence would wait for every
// outstanding LDS fill); ordering of the fills is by wait_vmcnt.
__device__ __forceinline__ void barrier_only()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One slice of MFMAs from a stage.  Per slice of 16 along K a wave needs WTM
// A and WTN B fragments (8 bf16 per lane: row lane % 32, chunk
// 2 * slice + lane / 32); a K step reads both slices' fragments first and
// then runs both slices' MFMAs (fill_schedule orders the step).
template <int WTM, int WTN>
__device__ __forceinline__ void mfma_frags(const bf16x8 (&fa)[WTM], const bf16x8 (&fb)[WTN], f32x16 (&acc)[WTM][WTN])
{
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
        for (int c = 0; c < WTN; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[c], acc[a][c], 0, 0, 0);
}

template <int WTM, int WTN>
__device__ __forceinline__ void read_frags(const unsigned char *a_rows, const unsigned char *b_rows, int off,
                                           bf16x8 (&fa)[WTM], bf16x8 (&fb)[WTN])
{
#pragma unroll
    for (int a = 0; a < WTM; ++a) fa[a] = *reinterpret_cast<const bf16x8 *>(a_rows + a * 32 * 64 + off);
#pragma unroll
    for (int c = 0; c < WTN; ++c) fb[c] = *reinterpret_cast<const bf16x8 *>(b_rows + c * 32 * 64 + off);
}

// Buffer resource over a row panel of a BF16 matrix (raw addressing, no
// range clamp inside the panel): the fills address it with a per-lane
// 32-bit offset and a wave-uniform one, no 64-bit address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const uint16_t *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(base), (short)0, 0x7fffffff, 0x00020000);
}

// Fill stage `stage` with K step `step`: this wave's NB blocks (block
// wave + j * WAVES; A blocks first, then B), 16 rows each, from the row
// panels rA (A rows m0 ..) and rB (B rows n0 ..).  Lane i loads row i / 4
// of its block at byte offset voff (row and swizzled chunk); the block row
// and the step go in the uniform offset.
template <class S>
__device__ __forceinline__ void fill_stage(unsigned char *smem, __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rB,
                                           int row_bytes, int wave, int voff, int step, int stage)
{
    unsigned char *st = smem + (size_t)stage * S::STAGE;
#pragma unroll
    for (int j = 0; j < S::BLK_PER_WAVE; ++j) {
        const int blk = wave + j * S::WAVES;
        const bool in_a = blk < S::A_BLK;
        const int soff = (in_a ? blk : blk - S::A_BLK) * 16 * row_bytes + step * (kBK * 2);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(in_a ? rA : rB, (lds_void *)(st + blk * 1024), 16, voff, soff, 0, 0);
    }
}

template <int WGM, int WGN, int WTM, int WTN, int CAND>
__global__ __launch_bounds__(64 * WGM * WGN) void k_corr_topk(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                                        const float *__restrict__ norm2, int64_t Kp, int m_blocks,
                                                        int n_tiles, int tiles_per_seg, int n_seg, int gm, int gs,
                                                        int64_t col0, int list_stride, int list_base,
                                                        float *__restrict__ out_s, int32_t *__restrict__ out_i)
{
    using S = CorrShape<WGM, WGN, WTM, WTN>;
    constexpr int BM = S::BM, BN = S::BN, TPR = S::TPR, NB = S::BLK_PER_WAVE;
    static_assert(TPR >= 1 && S::THREADS % BM == 0, "tile too small for the workgroup");
    static_assert((BN / WGN) % 64 == 0, "each wave must own whole 64-column epilogue passes");
    static_assert(CAND == 16 || CAND == 32 || CAND == 64, "candidate lists of 16, 32 or 64");
    constexpr bool WAVE_LIST = CAND == 64;
    constexpr int RPW = S::RPW;
    extern __shared__ __align__(16) unsigned char smem[];
    float *Cs = reinterpret_cast<float *>(smem);                       // [BM][65], aliases the stages

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WGM, wn = wave / WGM;
    // XCD-aware ordering: workgroup ids are dealt round-robin to the 8 XCDs,
    // and each XCD takes a contiguous range u of an order of the (m_block,
    // seg) pairs that walks blocks of gm row blocks x gs segments: the
    // workgroups resident on one XCD at a time (about gm x gs) then stream
    // gm panels of ROI images and gs library segments through its L2
    // instead of one panel per workgroup.
    int mb, seg;
    {
        const int T = m_blocks * n_seg;
        const int x = blockIdx.x & 7, j = blockIdx.x >> 3;
        const int q = T >> 3, r = T & 7;
        const int u = x * q + min(x, r) + j;
        const int full = m_blocks / gm;                   // block rows of gm row blocks
        const int sm = min(u / (gm * n_seg), full);       // block row of u (the last may be short)
        const int rows = sm < full ? gm : m_blocks - full * gm;
        const int rem = u - sm * gm * n_seg;
        const int ss = rem / (rows * gs);                 // block column (the last may be narrow)
        const int l = rem - ss * rows * gs;
        mb = sm * gm + l % rows;
        seg = ss * gs + l / rows;
    }
    const int64_t m0 = (int64_t)mb * BM;
    const int t0 = seg * tiles_per_seg;
    const int t1 = min(t0 + tiles_per_seg, n_tiles);

    // fill side: wave-block j of a stage is block wave + j * WAVES (A blocks
    // first, then B); lane i loads row 16 * blk + i / 4, logical chunk
    // (i % 4) ^ ((i / 16) % 4), and lands at byte 16 i of the block
    const int row_bytes = (int)(Kp * 2);
    const int voff = (lane >> 2) * row_bytes + 16 * ((lane & 3) ^ ((lane >> 4) & 3));
    const __amdgpu_buffer_rsrc_t rA = panel_rsrc(A + m0 * Kp);
    // read side: fragment row (lane % 32) of every 32-row group, chunk
    // 2 * slice + lane / 32 stored at chunk ^ ((lane >> 2) & 3)
    const int r_x = (lane >> 2) & 3;
    const int r_off0 = (lane & 31) * 64 + 16 * ((lane >> 5) ^ r_x);
    const int r_off1 = (lane & 31) * 64 + 16 * ((2 + (lane >> 5)) ^ r_x);

    // epilogue ownership: thread -> (row, part of each 64-column pass)
    const int e_row = tid % BM;
    const int e_part = tid / BM;
    TopList<WAVE_LIST ? 1 : CAND> top;
    top.init();
    float wl_s[WAVE_LIST ? RPW : 1];   // 64-entry lists: rows wave + WAVES * j, entry `lane`
    int wl_i[WAVE_LIST ? RPW : 1];
#pragma unroll
    for (int j = 0; j < (WAVE_LIST ? RPW : 1); ++j) {
        wl_s[j] = INFINITY;
        wl_i[j] = 0x7fffffff;
    }

    const int KT = (int)(Kp / kBK);
    for (int nt = t0; nt < t1; ++nt) {
        const int64_t n0 = col0 + (int64_t)nt * BN;
        const __amdgpu_buffer_rsrc_t rB = panel_rsrc(B + n0 * Kp);
        f32x16 acc[WTM][WTN];
#pragma unroll
        for (int a = 0; a < WTM; ++a)
#pragma unroll
            for (int c = 0; c < WTN; ++c)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][c][r] = 0.0f;

        __syncthreads();   // the previous tile's epilogue read Cs, which aliases the stages
        // Every step issues exactly NB fills per wave, so the wait below is a
        // constant: steps past the end reload step KT - 1 into the stage the
        // previous step read (no later step reads it), and a K shorter than
        // the ring fills the spare stages with step KT - 1 as well.
#pragma unroll
        for (int p = 0; p < kStages - 1; ++p) fill_stage<S>(smem, rA, rB, row_bytes, wave, voff, min(p, KT - 1), p);
        for (int kt = 0; kt < KT; ++kt) {
            // this wave's fills of step kt have landed once at most the fills
            // of the kStages - 2 later steps in flight remain outstanding
            wait_vmcnt<(kStages - 2) * NB>();
            barrier_only();   // every wave's fills of step kt have landed; step kt - 1's stage is free
            const unsigned char *st = smem + (size_t)(kt % kStages) * S::STAGE;
            const unsigned char *a_rows = st + (wm * (BM / WGM)) * 64;
            const unsigned char *b_rows = st + S::A_BYTES + (wn * (BN / WGN)) * 64;
            bf16x8 fa0[WTM], fb0[WTN], fa1[WTM], fb1[WTN];
            read_frags<WTM, WTN>(a_rows, b_rows, r_off0, fa0, fb0);
            read_frags<WTM, WTN>(a_rows, b_rows, r_off1, fa1, fb1);
            mfma_frags<WTM, WTN>(fa0, fb0, acc);
            mfma_frags<WTM, WTN>(fa1, fb1, acc);
            fill_stage<S>(smem, rA, rB, row_bytes, wave, voff, min(kt + kStages - 1, KT - 1),
                          (kt + kStages - 1) % kStages);
            __builtin_amdgcn_sched_group_barrier(0x100, 2 * (WTM + WTN), 0);   // the fragment reads first
            fill_schedule<0, NB, 2 * WTM * WTN>();
        }
        wait_vmcnt<0>();   // the fills past the end land before Cs reuses the stages
        __syncthreads();
        // epilogue in 64-column passes: the waves owning the columns write their
        // scores |L|^2 - 2<S,L> to LDS, then every thread scans its share of a row
#pragma unroll
        for (int h = 0; h < BN / 64; ++h) {
            constexpr int WCOLS = BN / WGN;               // columns per wave
            const int wave_of_pass = (h * 64) / WCOLS;    // compile-time after unrolling
            if (wn == wave_of_pass) {
                const int c0 = (h * 64 - wave_of_pass * WCOLS) / 32;   // first 32-wide tile of the pass
#pragma unroll
                for (int a = 0; a < WTM; ++a)
#pragma unroll
                    for (int c = 0; c < WTN; ++c) {
                        if (c == c0 || c == c0 + 1) {
                            const int col = (c - c0) * 32 + (lane & 31);
                            const float nrm = norm2[n0 + h * 64 + col];
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                const int row = wm * (BM / WGM) + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                                Cs[row * 65 + col] = fmaf(-2.0f, acc[a][c][r], nrm);
                            }
                        }
                    }
            }
            __syncthreads();
            if constexpr (WAVE_LIST) {
                const int col = (int)(n0 + h * 64) + lane;
#pragma unroll
                for (int j = 0; j < RPW; ++j)
                    wave_merge64(wl_s[j], wl_i[j], Cs[(wave + S::WAVES * j) * 65 + lane], col, lane);
            } else {
                constexpr int W = 64 / TPR;
                const float *crow = Cs + e_row * 65 + e_part * W;
                const int base = (int)(n0 + h * 64 + e_part * W);
#pragma unroll 1
                for (int j = 0; j < W; ++j) top.insert(crow[j], base + j);
            }
            __syncthreads();
        }
    }
    if constexpr (WAVE_LIST) {
#pragma unroll
        for (int j = 0; j < RPW; ++j) {
            const size_t o = (((size_t)(m0 + wave + S::WAVES * j)) * list_stride + list_base + seg) * CAND + lane;
            out_s[o] = wl_s[j];
            out_i[o] = wl_i[j];
        }
    } else {
        const size_t o = (((size_t)(m0 + e_row)) * list_stride + list_base + seg * TPR + e_part) * CAND;
#pragma unroll
        for (int j = 0; j < CAND; ++j) {
            out_s[o + j] = top.s[j];
            out_i[o + j] = top.i[j];
        }
    }
}

// Epilogue lists per row and segment of a tile configuration.
constexpr int lists_per_row(int cand, int threads, int bm) { return cand == 64 ? 1 : threads / bm; }

// ------------------------------------------------------------ merge
// One wave per row: the CAND smallest (score, index) over n_lists lists.
template <int CAND>
__global__ __launch_bounds__(256) void k_merge(const float *__restrict__ in_s, const int32_t *__restrict__ in_i,
                                               int n_lists, int64_t n_rows, int32_t *__restrict__ cand_idx)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int n = n_lists * CAND;
    const float *s = in_s + (size_t)row * n;
    const int32_t *ix = in_i + (size_t)row * n;
    // each lane keeps its private best CAND of the strided elements
    TopList<CAND> t;
    t.init();
    for (int e = lane; e < n; e += 64) t.insert(s[e], ix[e]);
    wave_select<CAND>(t, [&](int j, float, int bi) {
        if (lane == 0) cand_idx[(size_t)row * CAND + j] = bi;
    });
}

// One wave per row, 64 candidates: the lists are read 64 entries at a time
// and merged into one wave-wide list.
__global__ __launch_bounds__(256) void k_merge64(const float *__restrict__ in_s, const int32_t *__restrict__ in_i,
                                                 int n_lists, int64_t n_rows, int32_t *__restrict__ cand_idx)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int n = n_lists * 64;
    const float *s = in_s + (size_t)row * n;
    const int32_t *ix = in_i + (size_t)row * n;
    float ls = INFINITY;
    int li = 0x7fffffff;
    for (int e = 0; e < n; e += 64) wave_merge64(ls, li, s[e + lane], ix[e + lane], lane);
    cand_idx[(size_t)row * 64 + lane] = li;
}

// ------------------------------------------------------------ FP32 rescore
// One workgroup per ROI row: Delta for each candidate from the FP32 images,
// then the k best by (Delta, index).
template <int CAND, bool STAGE>
__global__ __launch_bounds__(256) void k_rescore(const float *__restrict__ S, const float *__restrict__ inv_s,
                                                 const float *__restrict__ L, const float *__restrict__ inv_l,
                                                 const int32_t *__restrict__ cand_idx, int n_win, int n_dir,
                                                 int64_t n_lib, int k, int32_t *__restrict__ top_idx,
                                                 float *__restrict__ top_score)
{
#pragma clang fp contract(off)
    extern __shared__ float stage[];
    __shared__ float ds[CAND];
    __shared__ int di[CAND];
    constexpr int PER = CAND / 4;   // candidates per wave
    const int64_t r = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float *srow = S + (size_t)r * n_win * n_dir;
    int cl[PER];
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int l = cand_idx[(size_t)r * CAND + wave + 4 * q];
        cl[q] = (l >= 0 && l < n_lib) ? l : -1;
        acc[q] = 0.0f;
    }
    for (int w = 0; w < n_win; ++w) {
        const float is = inv_s[(size_t)r * n_win + w];
        const float *src = srow + (size_t)w * n_dir;
        if (STAGE) {
            __syncthreads();
            // the ROI's normalised window, sixteen loads in flight per thread
            for (int v0 = threadIdx.x; v0 < n_dir; v0 += 256 * 16) {
                float x[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) x[e] = v0 + 256 * e < n_dir ? src[v0 + 256 * e] : 0.0f;
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (v0 + 256 * e < n_dir) stage[v0 + 256 * e] = x[e] * is;
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (cl[q] < 0) continue;
            const float il = inv_l[(size_t)cl[q] * n_win + w];
            const float *lrow = L + ((size_t)cl[q] * n_win + w) * n_dir;
#pragma unroll 8
            for (int v = lane; v < n_dir; v += 64) {
                // both normalised values rounded alike (no contraction in this
                // kernel): identical images give Delta = 0 exactly
                const float a = STAGE ? stage[v] : src[v] * is;
                const float d = a - lrow[v] * il;
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
            ds[wave + 4 * q] = cl[q] >= 0 ? a : INFINITY;
            di[wave + 4 * q] = cl[q] >= 0 ? cl[q] : 0x7fffffff;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // insertion sort of CAND entries by (Delta, index)
        for (int a = 1; a < CAND; ++a) {
            const float vs = ds[a];
            const int vi = di[a];
            int b = a - 1;
            while (b >= 0 && (ds[b] > vs || (ds[b] == vs && di[b] > vi))) {
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

// The ROI window is staged in LDS when n_dir floats fit beside the static
// arrays; otherwise both rows are read from global memory.
template <int CAND>
ar_status launch_rescore(ar_context *ctx, const float *images, const ar_library *lib, int64_t n_roi, int k,
                         int32_t *top_idx, float *top_score, hipStream_t s)
{
    const size_t stage = sizeof(float) * (size_t)lib->n_dir;
    if (stage + 4096 <= (size_t)ctx->lds_per_block) {
        if (stage > 65536)   // on every launch: the attribute belongs to the current device
            AR_HIP(hipFuncSetAttribute((const void *)k_rescore<CAND, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)stage));
        k_rescore<CAND, true><<<(unsigned)n_roi, 256, stage, s>>>(images, ctx->i_inv.as<float>(), lib->ref,
                                                                  lib->inv_max.as<float>(),
                                                                  ctx->i_merge_idx.as<int32_t>(), lib->n_win,
                                                                  lib->n_dir, lib->n_lib, k, top_idx, top_score);
    } else {
        k_rescore<CAND, false><<<(unsigned)n_roi, 256, 0, s>>>(images, ctx->i_inv.as<float>(), lib->ref,
                                                               lib->inv_max.as<float>(),
                                                               ctx->i_merge_idx.as<int32_t>(), lib->n_win,
                                                               lib->n_dir, lib->n_lib, k, top_idx, top_score);
    }
    AR_HIP(hipGetLastError());
    return AR_OK;
}

// Orientation and phase of library entries idx[i] (-1 or out of range: NaN
// quaternion, phase -1).
__global__ __launch_bounds__(256) void k_library_lookup(const double *__restrict__ lq, const int32_t *__restrict__ lp,
                                                        int64_t n_lib, const int32_t *__restrict__ idx, int64_t n,
                                                        double *__restrict__ quats, int32_t *__restrict__ phase)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t l = idx[i];
    const bool ok = l >= 0 && l < n_lib;
    if (quats)
        for (int c = 0; c < 4; ++c) quats[4 * i + c] = ok ? lq[4 * (int64_t)l + c] : __builtin_nan("");
    if (phase) phase[i] = ok ? lp[l] : -1;
}

template <int CAND>
__global__ void k_copy_cand(const int32_t *__restrict__ cand, int64_t n_rows, int32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_rows * CAND) out[i] = cand[i];
}

// Correlation tile configurations: WAVES 4 (2x2 wave grid) or 8 (2x4), per-wave
// 32x32 tiles WTM x WTN, K step BK.
struct CorrCfg {
    int waves, wtm, wtn, bk;
    int wgn() const { return waves == 8 ? 4 : 2; }
    int bm() const { return 32 * wtm * 2; }
    int bn() const { return 32 * wtn * wgn(); }
    int threads() const { return 64 * waves; }
    // dynamic LDS of the tile (CorrShape::lds)
    size_t lds() const
    {
        const size_t ab = (size_t)kStages * (bm() + bn()) * kBK * 2, c = (size_t)bm() * 65 * sizeof(float);
        return ab > c ? ab : c;
    }
};

// One correlation launch over the library rows [col0, col0 + n_tiles * BN).
struct CorrLaunch {
    int m_blocks, n_tiles, tiles_per_seg, n_seg;
    int64_t col0;
    int list_stride, list_base;
    int gm = 1, gs = 1;   // XCD blocking: row blocks x segments walked together (set by launch_corr_t)
};

// Blocking of the (row block, segment) pairs for the workgroups resident on
// one XCD at a time (`resident`): gs segments (at most 8) by gm row blocks.
void xcd_blocking(int m_blocks, int n_seg, int resident, int &gm, int &gs)
{
    gs = std::max(1, std::min(n_seg, 8));
    gm = std::max(1, std::min(m_blocks, resident / gs));
}

template <int WGM, int WGN, int WTM, int WTN, int CAND>
ar_status launch_corr_t(ar_context *ctx, const uint16_t *A, const ar_library *lib, const CorrLaunch &L,
                        float *out_s, int32_t *out_i, hipStream_t s)
{
    const int m_blocks = L.m_blocks, n_tiles = L.n_tiles, tiles_per_seg = L.tiles_per_seg, n_seg = L.n_seg;
    using S = CorrShape<WGM, WGN, WTM, WTN>;
    const unsigned blocks = (unsigned)(m_blocks * n_seg);
    const size_t lds = S::lds();
    AR_CHECK((size_t)ctx->lds_per_block >= lds, "correlation tile needs %zu bytes of LDS per workgroup", lds);
    if (lds > 65536)   // on every launch: the attribute belongs to the current device
        AR_HIP(hipFuncSetAttribute((const void *)k_corr_topk<WGM, WGN, WTM, WTN, CAND>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int per_cu = std::max(1, std::min((int)(ctx->lds_per_block / lds), 8 / S::WAVES));
    int gm, gs;
    xcd_blocking(m_blocks, n_seg, per_cu * ctx->cu_count / 8, gm, gs);
    k_corr_topk<WGM, WGN, WTM, WTN, CAND><<<blocks, S::THREADS, lds, s>>>(
        A, lib->bf16.as<uint16_t>(), lib->norm2.as<float>(), lib->Kp, m_blocks, n_tiles, tiles_per_seg, n_seg, gm, gs,
        L.col0, L.list_stride, L.list_base, out_s, out_i);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

// (waves, wtm, wtn): 2x2 or 2x4 wave grids, K step 32
#define AR_CORR_TILES(X) X(4, 2, 2) X(4, 2, 4) X(4, 4, 2) X(4, 4, 4) X(8, 2, 2) X(8, 4, 2)

bool corr_tile_supported(int waves, int wtm, int wtn, int bk)
{
#define AR_CORR_IS(w_, m_, n_) if (waves == w_ && wtm == m_ && wtn == n_ && bk == kBK) return true;
    AR_CORR_TILES(AR_CORR_IS)
#undef AR_CORR_IS
    return false;
}

template <int CAND>
ar_status launch_corr(ar_context *ctx, const CorrCfg &c, const uint16_t *A, const ar_library *lib,
                      const CorrLaunch &L, float *out_s, int32_t *out_i, hipStream_t s)
{
#define AR_CORR_CASE(w_, m_, n_)                                                                   \
    if (c.waves == w_ && c.wtm == m_ && c.wtn == n_)                                               \
        return launch_corr_t<2, (w_) / 2, m_, n_, CAND>(ctx, A, lib, L, out_s, out_i, s);
    AR_CORR_TILES(AR_CORR_CASE)
#undef AR_CORR_CASE
    return fail(AR_EINVAL, "unsupported correlation tile %d waves %dx%dx%d", c.waves, c.wtm, c.wtn, c.bk);
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Normalise FP32 images [n][n_win][n_dir] into a BF16 [n_pad][Kp] matrix and
// FP32 reciprocal maxima [n][n_win].
ar_status normalise_cast(const float *img, int64_t n, int64_t n_pad, int n_win, int n_dir, int64_t Kp, float *inv,
                         uint16_t *out, hipStream_t s)
{
    dim3 grid((unsigned)n, (unsigned)n_win);
    k_normalise_cast<<<grid, 256, 0, s>>>(img, n_win, n_dir, Kp, inv, out);
    AR_HIP(hipGetLastError());
    if (n_pad > n) {
        k_zero_rows<<<256, 256, 0, s>>>(out, Kp, n, n_pad);
        AR_HIP(hipGetLastError());
    }
    return AR_OK;
}

// Correlation (main and optional tail launch), merge, FP32 rescore and the
// optional copy of the BF16-stage candidates, for CAND candidates per row.
template <int CAND>
ar_status run_index(ar_context *ctx, const CorrCfg &cfg, const CorrCfg &tail_cfg, bool split, const CorrLaunch &main_l,
                    const CorrLaunch &tail_l, int n_lists, const float *images, const ar_library *lib, int64_t n_roi,
                    int k, int32_t *top_idx, float *top_score, int32_t *cand_idx, hipStream_t s)
{
    const uint16_t *A = ctx->i_bf16.as<uint16_t>();
    float *cs = ctx->i_cand_score.as<float>();
    int32_t *ci = ctx->i_cand_idx.as<int32_t>();
    int32_t *merged = ctx->i_merge_idx.as<int32_t>();
    AR_TRY(launch_corr<CAND>(ctx, cfg, A, lib, main_l, cs, ci, s));
    if (split) AR_TRY(launch_corr<CAND>(ctx, tail_cfg, A, lib, tail_l, cs, ci, s));
    if constexpr (CAND == 64)
        k_merge64<<<(unsigned)((n_roi + 3) / 4), 256, 0, s>>>(cs, ci, n_lists, n_roi, merged);
    else
        k_merge<CAND><<<(unsigned)((n_roi + 3) / 4), 256, 0, s>>>(cs, ci, n_lists, n_roi, merged);
    AR_HIP(hipGetLastError());
    AR_TRY(launch_rescore<CAND>(ctx, images, lib, n_roi, k, top_idx, top_score, s));
    if (cand_idx) {
        const int64_t n = n_roi * CAND;
        k_copy_cand<CAND><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(merged, n_roi, cand_idx);
        AR_HIP(hipGetLastError());
    }
    return AR_OK;
}

}  // namespace idx
}  // namespace ar

using namespace ar;

extern "C" {

ar_status ar_library_create(ar_context *ctx, const float *ref_images, int64_t n_lib, int32_t n_win, int32_t n_dir,
                            void *stream, ar_library **out)
{
    AR_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(ref_images != nullptr, "ref_images is NULL");
    AR_CHECK(n_lib >= 1 && n_lib < (int64_t)INT32_MAX - idx::kPadN, "n_lib out of range");
    AR_CHECK(n_win >= 1 && n_dir >= 1, "n_win and n_dir must be >= 1");
    // the correlation addresses a 256-row panel of BF16 rows with 32-bit byte offsets
    AR_CHECK(idx::round_up((int64_t)n_win * n_dir, idx::kPadK) * 2 * 256 < (int64_t)INT32_MAX,
             "n_win * n_dir = %lld too large (at most %d)", (long long)n_win * n_dir, (int)(INT32_MAX / 512) & ~63);
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    auto *lib = new (std::nothrow) ar_library();
    if (!lib) return fail(AR_ENOMEM, "library allocation failed");
    lib->ctx = ctx;
    lib->ref = ref_images;
    lib->n_lib = n_lib;
    lib->n_win = n_win;
    lib->n_dir = n_dir;
    lib->K = (int64_t)n_win * n_dir;
    lib->Kp = idx::round_up(lib->K, idx::kPadK);
    lib->n_pad = idx::round_up(n_lib, idx::kPadN);
    ar_status st = lib->bf16.reserve(sizeof(uint16_t) * (size_t)lib->n_pad * lib->Kp);
    if (st == AR_OK) st = lib->norm2.reserve(sizeof(float) * lib->n_pad);
    if (st == AR_OK) st = lib->inv_max.reserve(sizeof(float) * n_lib * n_win);
    if (st == AR_OK)
        st = idx::normalise_cast(ref_images, n_lib, lib->n_pad, n_win, n_dir, lib->Kp, lib->inv_max.as<float>(),
                                 lib->bf16.as<uint16_t>(), s);
    if (st == AR_OK) {
        idx::k_row_norm2<<<(unsigned)lib->n_pad, 256, 0, s>>>(lib->bf16.as<uint16_t>(), lib->Kp, n_lib,
                                                              lib->norm2.as<float>());
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = fail(AR_EDEVICE, "k_row_norm2: %s", hipGetErrorString(e));
    }
    if (st != AR_OK) {
        delete lib;
        return st;
    }
    *out = lib;
    return AR_OK;
}

ar_status ar_library_prepare(ar_context *ctx, const float *ref_images, int64_t n_lib, int32_t n_win, int32_t n_dir,
                             const double *quats, const int32_t *phase, void *stream, ar_library **out)
{
    AR_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    AR_CHECK(quats && phase, "quats/phase must not be NULL (ar_library_create takes images alone)");
    ar_library *lib = nullptr;
    AR_TRY(ar_library_create(ctx, ref_images, n_lib, n_win, n_dir, stream, &lib));
    ar_status st = lib->quats.reserve(sizeof(double) * 4 * (size_t)n_lib);
    if (st == AR_OK) st = lib->phase.reserve(sizeof(int32_t) * (size_t)n_lib);
    hipStream_t s = (hipStream_t)stream;
    if (st == AR_OK) {
        hipError_t e = hipMemcpyAsync(lib->quats.ptr, quats, sizeof(double) * 4 * (size_t)n_lib,
                                      hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lib->phase.ptr, phase, sizeof(int32_t) * (size_t)n_lib, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = fail(AR_EDEVICE, "copying the orientations: %s", hipGetErrorString(e));
    }
    if (st != AR_OK) {
        ar_library_destroy(lib);
        return st;
    }
    lib->has_orientations = true;
    *out = lib;
    return AR_OK;
}

ar_status ar_library_lookup(const ar_library *lib, const int32_t *idx, int64_t n, double *quats, int32_t *phase,
                            void *stream)
{
    AR_CHECK(lib != nullptr, "library is NULL");
    AR_CHECK(lib->has_orientations, "library was created without orientations (use ar_library_prepare)");
    AR_CHECK(n >= 0, "n must be >= 0");
    if (n == 0) return AR_OK;
    AR_CHECK(idx != nullptr && (quats || phase), "idx is NULL or no output given");
    AR_CHECK((n + 255) / 256 < (int64_t)INT32_MAX, "too many entries");
    AR_HIP(hipSetDevice(lib->ctx->device));
    idx::k_library_lookup<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        lib->quats.as<double>(), lib->phase.as<int32_t>(), lib->n_lib, idx, n, quats, phase);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

ar_status ar_library_destroy(ar_library *lib)
{
    if (!lib) return AR_OK;
    (void)hipSetDevice(lib->ctx->device);
    (void)hipDeviceSynchronize();
    delete lib;
    return AR_OK;
}

ar_status index_orientations_ex(ar_context *ctx, const float *images, int64_t n_roi, const ar_library *lib, int32_t k,
                                int32_t cand, int32_t *top_idx, float *top_score, int32_t *cand_idx, void *stream)
{
    AR_CHECK(ctx && lib, "ctx/library is NULL");
    AR_CHECK(images && top_idx && top_score, "images/top_idx/top_score must not be NULL");
    AR_CHECK(n_roi >= 1 && n_roi < (int64_t)INT32_MAX - idx::kPadM, "n_roi out of range");
    AR_CHECK(cand == 16 || cand == 32 || cand == 64, "cand must be 16, 32 or 64, got %d", cand);
    AR_CHECK(k >= 1 && k <= cand, "k must be in [1, cand = %d], got %d", cand, k);
    AR_CHECK(lib->ctx == ctx, "library belongs to another context");
    AR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // Default tile: 256 x 256 (8 waves of 4 x 2 MFMA tiles).  Longer
    // candidate lists (cand = 32 per thread, 64 per wave) do not fit beside
    // the 8-wave tile's accumulators, so cand >= 32 takes the same 256 x 256
    // tile on 4 waves of 4 x 4 MFMA tiles (one wave per SIMD, 512 registers
    // each), with identical results.  Measured, ms per call (128 x 256 on 8
    // waves / 256 x 256 on 4): k = 32: 6.5 / 5.4 at 2000 x 20000, 15.6 / 12.7
    // at 5000 x 20000, 238 / 173 at 20000 x 100000; k = 64: 8.0 / 7.7, 19.0 /
    // 18.0, 254 / 225.  A 16-candidate call whose segments (planned below,
    // the same for both 256 x 256 forms) walk at least 6 tiles takes the
    // 4-wave form too: its K loop is faster, its epilogue (one thread per
    // row) slower, and long segments keep the lists' insertions rare.
    // Measured (ms per call, 8 waves / 4 waves): 20000 x 100000 (25 tiles
    // per segment) 166.1-167.7 / 159.9-160.3; 2500 x 100000 (16) 20.5-20.6
    // / 18.7; 5000 x 20000 (7) 10.5 / 9.8; 10000 x 40000 (5) 33.7-33.8 /
    // 34.2; 20000 x 12500 (2) 27.6-27.8 / 28.0.
    const int64_t m_pad = idx::round_up(n_roi, idx::kPadM);
    idx::CorrCfg cfg = ctx->corr_tile_set ? idx::CorrCfg{ctx->corr_waves, ctx->corr_wtm, ctx->corr_wtn, ctx->corr_bk}
                       : cand >= 32       ? idx::CorrCfg{4, 4, 4, idx::kBK}
                                          : idx::CorrCfg{8, 4, 2, idx::kBK};
    const int m_blocks = (int)(m_pad / cfg.bm());
    const int n_tiles = (int)(lib->n_pad / cfg.bn());
    // segments: a workgroup walks tiles_per_seg column tiles of one row block.
    // The makespan is rounds of resident workgroups times tiles per
    // workgroup (workgroups per CU from LDS and the 8 waves a CU holds at
    // this register budget); the fewest segments within 5 % of the best
    // makespan keep the candidate lists short.
    int tiles_per_seg = n_tiles, n_seg = 1;
    auto per_cu_of = [&](const idx::CorrCfg &c) {
        return std::max(1, std::min((int)(ctx->lds_per_block / c.lds()), 8 / c.waves));
    };
    const int per_cu = per_cu_of(cfg);
    const int64_t slots = (int64_t)per_cu * ctx->cu_count;
    {
        auto makespan = [&](int ns, int &tps, int &nsr) {
            tps = (n_tiles + ns - 1) / ns;
            nsr = (n_tiles + tps - 1) / tps;
            return ((int64_t)m_blocks * nsr + slots - 1) / slots * tps;
        };
        int64_t best = INT64_MAX;
        for (int ns = 1; ns <= n_tiles; ++ns) {
            int tps, nsr;
            best = std::min(best, makespan(ns, tps, nsr));
        }
        for (int ns = 1; ns <= n_tiles; ++ns) {
            int tps, nsr;
            if (makespan(ns, tps, nsr) * 100 <= best * 105) {
                tiles_per_seg = tps;
                n_seg = nsr;
                break;
            }
        }
    }
    if (!ctx->corr_tile_set && cand == 16 && tiles_per_seg >= 6) cfg = idx::CorrCfg{4, 4, 4, idx::kBK};
    // One-tile segments whose last round is partial (small calls): the whole
    // rounds run the main tile and the remaining columns a tile of the same
    // height and half the width (4 waves), all in one more round.  Every
    // score accumulates K in the same order in either tile, so the candidate
    // lists are the same as from the main tile alone.
    // Taken when its makespan, the whole rounds plus 0.75 of a main tile (the
    // half-width tile runs at 4 waves per CU; measured ~0.7), beats the
    // segmented one.
    idx::CorrLaunch main_l{m_blocks, n_tiles, tiles_per_seg, n_seg, 0, 0, 0}, tail_l{};
    const idx::CorrCfg tail_cfg{4, cfg.wtm, cfg.wtn, cfg.bk};
    bool split = false;
    {
        const int64_t wgs = (int64_t)m_blocks * n_tiles;   // one tile per workgroup
        const int64_t seg_cost = ((int64_t)m_blocks * n_seg + slots - 1) / slots * tiles_per_seg;
        if (per_cu == 1 && cfg.waves == 8 && tail_cfg.bm() == cfg.bm() && 2 * tail_cfg.bn() == cfg.bn() &&
            idx::corr_tile_supported(4, cfg.wtm, cfg.wtn, cfg.bk) && wgs > slots && wgs % slots != 0 &&
            (wgs / slots) * 4 + 3 < seg_cost * 4) {
            const int main_cols = (int)((wgs / slots) * slots / m_blocks);
            const int tail_tiles = 2 * (n_tiles - main_cols);
            if (main_cols >= 1 && (int64_t)m_blocks * tail_tiles <= (int64_t)per_cu_of(tail_cfg) * ctx->cu_count) {
                split = true;
                main_l = idx::CorrLaunch{m_blocks, main_cols, 1, main_cols, 0, 0, 0};
                tail_l = idx::CorrLaunch{m_blocks, tail_tiles, 1, tail_tiles, (int64_t)main_cols * cfg.bn(), 0,
                                         main_cols * idx::lists_per_row(cand, cfg.threads(), cfg.bm())};
            }
        }
    }
    const int n_lists = main_l.n_seg * idx::lists_per_row(cand, cfg.threads(), cfg.bm()) +
                        (split ? tail_l.n_seg * idx::lists_per_row(cand, tail_cfg.threads(), tail_cfg.bm()) : 0);
    main_l.list_stride = tail_l.list_stride = n_lists;

    AR_TRY(ctx->i_bf16.reserve(sizeof(uint16_t) * (size_t)m_pad * lib->Kp));
    AR_TRY(ctx->i_inv.reserve(sizeof(float) * (size_t)n_roi * lib->n_win));
    AR_TRY(ctx->i_cand_score.reserve(sizeof(float) * (size_t)m_pad * n_lists * cand));
    AR_TRY(ctx->i_cand_idx.reserve(sizeof(int32_t) * (size_t)m_pad * n_lists * cand));
    AR_TRY(ctx->i_merge_idx.reserve(sizeof(int32_t) * (size_t)n_roi * cand));

    AR_TRY(idx::normalise_cast(images, n_roi, m_pad, lib->n_win, lib->n_dir, lib->Kp, ctx->i_inv.as<float>(),
                               ctx->i_bf16.as<uint16_t>(), s));
    switch (cand) {
    case 16: AR_TRY(idx::run_index<16>(ctx, cfg, tail_cfg, split, main_l, tail_l, n_lists, images, lib, n_roi, k, top_idx,
                                       top_score, cand_idx, s)); break;
    case 32: AR_TRY(idx::run_index<32>(ctx, cfg, tail_cfg, split, main_l, tail_l, n_lists, images, lib, n_roi, k, top_idx,
                                       top_score, cand_idx, s)); break;
    default: AR_TRY(idx::run_index<64>(ctx, cfg, tail_cfg, split, main_l, tail_l, n_lists, images, lib, n_roi, k, top_idx,
                                       top_score, cand_idx, s)); break;
    }
    return AR_OK;
}

ar_status ar_index_set_tile(ar_context *ctx, int32_t waves, int32_t wtm, int32_t wtn, int32_t bk)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    if (waves == 0 && wtm == 0 && wtn == 0 && bk == 0) {   // back to the default choice per candidate count
        ctx->corr_tile_set = false;
        return AR_OK;
    }
    AR_CHECK(idx::corr_tile_supported(waves, wtm, wtn, bk), "unsupported correlation tile %d waves %dx%dx%d", waves,
             wtm, wtn, bk);
    ctx->corr_waves = waves;
    ctx->corr_wtm = wtm;
    ctx->corr_wtn = wtn;
    ctx->corr_bk = bk;
    ctx->corr_tile_set = true;
    return AR_OK;
}

ar_status index_orientations(ar_context *ctx, const float *images, int64_t n_roi, const ar_library *lib, int32_t k,
                             int32_t *top_idx, float *top_score, void *stream)
{
    const int cand = k <= 16 ? 16 : k <= 32 ? 32 : 64;
    return index_orientations_ex(ctx, images, n_roi, lib, k, cand, top_idx, top_score, nullptr, stream);
}

}  // extern "C"
