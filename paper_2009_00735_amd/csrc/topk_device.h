// Device helpers for keeping the CAND smallest (score, index) pairs, shared
// by the dense and the sparse indexing kernels.  Order: ascending score,
// equal scores by ascending index.
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

}  // namespace ar
