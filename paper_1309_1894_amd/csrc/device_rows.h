// device_rows.h -- per-row work shared by the single-matrix row-block
// kernel and the batched tile kernel, so that a row gives the same bits in
// either.
#pragma once

#include "device_common.h"

namespace spk {

// Row stream of a run of short rows [r0, r1) whose entries [k0, k1) fit
// the LDS tile (k1 - k0 <= TILE, r1 - r0 <= 2*BS):
//   1. every lane issues its TILE/BS value and column loads at once
//      (coalesced: lane t takes entries k0 + t + j*BS), then the x gathers,
//      and stores the products in LDS; the run's row offsets go to LDS too;
//   2. each lane sums one row's products from LDS (two interleaved partial
//      sums) and writes y (and w = alpha*y + x).
// Products are rounded once (FP32 operands: exactly) and summed in FP64.
template <typename T, int BS, int TILE>
__device__ __forceinline__ void stream_rows(const int32_t *rp, const int32_t *ci, const T *val, const T *x,
                                            T *y, T *w, T alpha, int r0, int r1, int k0, int k1, double *sp,
                                            int *srp)
{
    constexpr int ITEMS = TILE / BS;
    static_assert(ITEMS * BS == TILE, "TILE must be a multiple of BS");
    const int t = threadIdx.x;
    const int nr = r1 - r0;
    const int nk = k1 - k0;
    for (int i = t; i <= nr; i += BS) srp[i] = rp[r0 + i] - k0;
    T v[ITEMS];
    int c[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = t + j * BS;
        v[j] = k < nk ? val[k0 + k] : T(0);
        c[j] = k < nk ? ci[k0 + k] : -1;
    }
    T xv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) xv[j] = c[j] >= 0 ? x[c[j]] : T(0);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = t + j * BS;
        if (k < nk) sp[k] = (double)v[j] * (double)xv[j];
    }
    __syncthreads();
    for (int i = t; i < nr; i += BS) {
        const int s = srp[i], e = srp[i + 1];
        double a0 = 0.0, a1 = 0.0;
        int k = s;
        for (; k + 1 < e; k += 2) {
            a0 += sp[k];
            a1 += sp[k + 1];
        }
        if (k < e) a0 += sp[k];
        const T yt = (T)(a0 + a1);
        y[r0 + i] = yt;
        if (w) w[r0 + i] = fma_t(alpha, yt, x[r0 + i]);
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
