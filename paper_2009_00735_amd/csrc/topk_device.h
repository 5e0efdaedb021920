// Device helpers for keeping the CAND smallest (score, index) pairs, shared
// by the dense and the sparse indexing kernels: per-thread sorted lists in
// registers (CAND 16, 32) and a wave-wide list of 64.  Order: ascending
// score, equal scores by ascending index.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ar {

__device__ __forceinline__ bool pair_less(float as, int ai, float bs, int bi)
{
    return as < bs || (as == bs && ai < bi);
}

// Sorted ascending by (score, index); insertion keeps the CAND smallest.
template <int CAND>
struct TopList {
    float s[CAND];
    int i[CAND];
    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int j = 0; j < CAND; ++j) {
            s[j] = INFINITY;
            i[j] = 0x7fffffff;
        }
    }
    __device__ __forceinline__ void insert(float cs, int ci)
    {
        if (!pair_less(cs, ci, s[CAND - 1], i[CAND - 1])) return;
#pragma unroll
        for (int j = 0; j < CAND; ++j) {
            const bool lt = pair_less(cs, ci, s[j], i[j]);
            const float ts = lt ? s[j] : cs;
            const int ti = lt ? i[j] : ci;
            s[j] = lt ? cs : s[j];
            i[j] = lt ? ci : i[j];
            cs = ts;
            ci = ti;
        }
    }
    // entry `head` (INFINITY past the end), selected without dynamic indexing
    __device__ __forceinline__ void at(int head, float &hs, int &hi) const
    {
        hs = INFINITY;
        hi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < CAND; ++q)
            if (q == head) {
                hs = s[q];
                hi = i[q];
            }
    }
};

// Wave-wide minimum of (score, index) pairs (64 lanes, butterfly).
__device__ __forceinline__ void wave_min_pair(float &bs, int &bi)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float os = __shfl_xor(bs, off);
        const int oi = __shfl_xor(bi, off);
        if (pair_less(os, oi, bs, bi)) {
            bs = os;
            bi = oi;
        }
    }
}

// The wave's CAND smallest pairs over every lane's sorted list t (each list
// holds at most CAND valid entries): CAND rounds of an argmin over the list
// heads.  Round j's result is passed to emit(j, score, index) on every lane.
template <int CAND, int LEN, typename Emit>
__device__ __forceinline__ void wave_select(const TopList<LEN> &t, Emit emit)
{
    int head = 0;
    for (int j = 0; j < CAND; ++j) {
        float hs;
        int hi;
        t.at(head, hs, hi);
        float bs = hs;
        int bi = hi;
        wave_min_pair(bs, bi);
        if (hs == bs && hi == bi && head < LEN) ++head;
        emit(j, bs, bi);
    }
}

// ---------------------------------------------------------------------------
// Wave-wide sorted list of 64 (score, index) pairs: lane j holds the j-th
// smallest.  A batch of 64 new pairs (one per lane) enters by a bitonic
// merge: the batch is sorted ascending across the lanes, reversed and
// combined lane by lane with the list by min (which leaves the 64 smallest
// of the 128 as a bitonic sequence), then sorted by the six half-cleaner
// steps.  Keys (score, index) are distinct except for the empty-slot
// sentinel, so the result is the exact 64 smallest whatever the order of
// arrival.

// Compare-exchange with the lane at distance `mask`: keep the smaller pair
// if keep_min, else the larger.
__device__ __forceinline__ void wave_cmpx(float &s, int &i, int mask, bool keep_min)
{
    const float os = __shfl_xor(s, mask);
    const int oi = __shfl_xor(i, mask);
    const bool other_less = pair_less(os, oi, s, i);
    if (keep_min == other_less) {
        s = os;
        i = oi;
    }
}

// Sort one pair per lane ascending across the 64 lanes.
__device__ __forceinline__ void wave_sort64(float &s, int &i, int lane)
{
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) wave_cmpx(s, i, j, ((lane & j) == 0) == ((lane & k) == 0));
}

// Merge the batch (bs, bi) into the sorted list (ls, li).  Lanes whose pair
// does not beat the list's last entry are dropped first; when none does,
// the list is unchanged and the merge is skipped.
__device__ __forceinline__ void wave_merge64(float &ls, int &li, float bs, int bi, int lane)
{
    const float ts = __shfl(ls, 63);
    const int ti = __shfl(li, 63);
    const bool enters = pair_less(bs, bi, ts, ti);
    if (!__any(enters)) return;
    if (!enters) {
        bs = INFINITY;
        bi = 0x7fffffff;
    }
    wave_sort64(bs, bi, lane);
    const float rs = __shfl(bs, 63 - lane);
    const int ri = __shfl(bi, 63 - lane);
    if (pair_less(rs, ri, ls, li)) {
        ls = rs;
        li = ri;
    }
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) wave_cmpx(ls, li, j, (lane & j) == 0);
}

}  // namespace ar
