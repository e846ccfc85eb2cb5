// device_rows.h -- per-row work shared by the single-matrix row-block
// kernel and the batched tile kernel, so that a row gives the same bits in
// either.
#pragma once

#include "device_common.h"

namespace spk {

// Row-stream of a run of short rows: stage values and gathered x of the
// run's entries in LDS with coalesced loads, then each lane sums one row in
// storage order.  Used by the row-block kernel and the batched kernel.
template <typename T, int BS, int TILE>
__device__ __forceinline__ void stream_rows(const int32_t *rp, const int32_t *ci, const T *val, const T *x,
                                            T *y, T *w, T alpha, int r0, int r1, T *sv, T *sx)
{
    const int t = threadIdx.x;
    const int k0 = rp[r0], k1 = rp[r1];
    for (int k = k0 + t; k < k1; k += BS) {
        sv[k - k0] = val[k];
        sx[k - k0] = x[ci[k]];
    }
    __syncthreads();
    for (int r = r0 + t; r < r1; r += BS) {
        const int s = rp[r] - k0, e = rp[r + 1] - k0;
        double acc = 0.0;
        for (int k = s; k < e; ++k) acc = fma_t((double)sv[k], (double)sx[k], acc);
        const T yt = (T)acc;
        y[r] = yt;
        if (w) w[r] = fma_t(alpha, yt, x[r]);
    }
    __syncthreads();
}

// G lanes per row over rows [r0, r1) of one matrix (all lanes take part).
template <typename T, int BS, int G>
__device__ __forceinline__ void group_rows(const int32_t *rp, const int32_t *ci, const T *val, const T *x,
                                           T *y, T *w, T alpha, int r0, int r1)
{
    constexpr int RPI = BS / G;
    const int t = threadIdx.x;
    const int lane = t & (G - 1);
    for (int rb = r0; rb < r1; rb += RPI) {
        const int row = rb + t / G;
        int s = 0, e = 0;
        if (row < r1) {
            s = rp[row];
            e = rp[row + 1];
        }
        double a0 = 0.0, a1 = 0.0;
        int k = s + lane;
        for (; k + G < e; k += 2 * G) {
            a0 = fma_t((double)val[k], (double)x[ci[k]], a0);
            a1 = fma_t((double)val[k + G], (double)x[ci[k + G]], a1);
        }
        if (k < e) a0 = fma_t((double)val[k], (double)x[ci[k]], a0);
        double sum = group_sum<G>(a0 + a1);
        if (lane == 0 && row < r1) {
            const T yt = (T)sum;
            y[row] = yt;
            if (w) w[row] = fma_t(alpha, yt, x[row]);
        }
    }
}

// One long row with the whole workgroup.
template <typename T, int BS>
__device__ __forceinline__ void block_row(const int32_t *rp, const int32_t *ci, const T *val, const T *x,
                                          T *y, T *w, T alpha, int row, double *red)
{
    const int t = threadIdx.x;
    const int s = rp[row], e = rp[row + 1];
    double a0 = 0.0, a1 = 0.0;
    int k = s + t;
    for (; k + BS < e; k += 2 * BS) {
        a0 = fma_t((double)val[k], (double)x[ci[k]], a0);
        a1 = fma_t((double)val[k + BS], (double)x[ci[k + BS]], a1);
    }
    if (k < e) a0 = fma_t((double)val[k], (double)x[ci[k]], a0);
    const double sum = block_sum<BS>(a0 + a1, red);
    if (t == 0) {
        const T yt = (T)sum;
        y[row] = yt;
        if (w) w[row] = fma_t(alpha, yt, x[row]);
    }
}

}  // namespace spk
