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
template <typename T, int BS, int TILE, int RG = 1>
__device__ __forceinline__ void stream_rows(const int32_t *rp, const int32_t *ci, const T *val, const T *x,
                                            T *y, T *w, T alpha, int r0, int r1, int k0, int k1, double *sp,
                                            int *srp)
{
    constexpr int ITEMS = TILE / BS;
    constexpr int RPT = kStreamRowsPerThread;
    static_assert(ITEMS * BS == TILE, "TILE must be a multiple of BS");
    const int t = threadIdx.x;
    const int nr = r1 - r0;
    const int nk = k1 - k0;
    // phase 1: every independent load of the run at once -- values,
    // columns, row offsets (and, for one lane per row, the x entries the
    // step adds to each row)
    T v[ITEMS];
    int c[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = t + j * BS;
        v[j] = k < nk ? val[k0 + k] : T(0);
        c[j] = k < nk ? ci[k0 + k] : -1;
    }
    int rpv[RPT + 1];
#pragma unroll
    for (int q = 0; q <= RPT; ++q) rpv[q] = (t + q * BS <= nr) ? rp[r0 + t + q * BS] - k0 : 0;
    T xo[RPT];
    if constexpr (RG == 1) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) xo[q] = (w && t + q * BS < nr) ? x[r0 + t + q * BS] : T(0);
    }
    // phase 2: the x gather, products to LDS
    T xv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) xv[j] = c[j] >= 0 ? x[c[j]] : T(0);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = t + j * BS;
        if (k < nk) sp[k] = (double)v[j] * (double)xv[j];
    }
#pragma unroll
    for (int q = 0; q <= RPT; ++q)
        if (t + q * BS <= nr) srp[t + q * BS] = rpv[q];
    __syncthreads();
    // phase 3: row sums from LDS
    if constexpr (RG == 1) {
        // one lane per row, two interleaved partial sums
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = t + q * BS;
            if (i < nr) {
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
                if (w) w[r0 + i] = fma_t(alpha, yt, xo[q]);
            }
        }
    } else {
        // RG adjacent lanes per row: they read consecutive LDS words (no
        // bank conflicts) and meet in a DPP group sum
        const int lane = t & (RG - 1);
        for (int rb = 0; rb < nr; rb += BS / RG) {
            const int i = rb + t / RG;
            double acc = 0.0;
            if (i < nr) {
                const int e = srp[i + 1];
                for (int k = srp[i] + lane; k < e; k += RG) acc += sp[k];
            }
            acc = group_sum<RG>(acc);
            if (lane == 0 && i < nr) {
                const T yt = (T)acc;
                y[r0 + i] = yt;
                if (w) w[r0 + i] = fma_t(alpha, yt, x[r0 + i]);
            }
        }
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

// ------------------------------------------------ wavefront-private tiles

// Orders a wavefront's own LDS writes before its later LDS reads: LDS
// operations of one wavefront execute in issue order, so only the compiler
// has to be kept from reordering them.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWaveTileRows = 2 * kWave;   // rows of one wavefront's row stream

// Products of a wavefront tile's entries, written to its LDS slice
// (sp[k - k0] for entry k).  Lane l takes entries k0 + l + 64j: coalesced
// 8-byte value and 4-byte column loads.
template <typename T, int ITEMS>
__device__ __forceinline__ void wave_products(const int32_t *ci, const T *val, const T *x, int k0, int nk, double *sp)
{
    const int l = threadIdx.x & (kWave - 1);
    T v[ITEMS];
    int c[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = l + j * kWave;
        // matrix entries are read exactly once: non-temporal, so the cache
        // keeps the x entries that neighbouring rows share
        v[j] = k < nk ? __builtin_nontemporal_load(val + k0 + k) : T(0);
        c[j] = k < nk ? __builtin_nontemporal_load(ci + k0 + k) : -1;
    }
    T xv[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) xv[j] = c[j] >= 0 ? x[c[j]] : T(0);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = l + j * kWave;
        if (k < nk) sp[k] = (double)v[j] * (double)xv[j];
    }
}

// One wavefront streams a run of short rows [r0, r1) with entries [k0, k1)
// (k1 - k0 <= 64*ITEMS, r1 - r0 <= 128) through its private LDS slice:
// all value/column/row-offset/own-x loads at once, then the x gather,
// products to LDS, one lane per row sums from LDS.  No workgroup barrier:
// every wavefront of a CU is an independent stream.
template <typename T, int ITEMS>
__device__ __forceinline__ void wave_stream(const int32_t *rp, const int32_t *ci, const T *val, const T *x, T *y,
                                            T *w, T alpha, int r0, int r1, int k0, int k1, double *sp, int *srp)
{
    const int l = threadIdx.x & (kWave - 1);
    const int nr = r1 - r0;
    const int nk = k1 - k0;
    int rpv[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) rpv[q] = (l + q * kWave <= nr) ? rp[r0 + l + q * kWave] - k0 : 0;
    T xo[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) xo[q] = (w && l + q * kWave < nr) ? x[r0 + l + q * kWave] : T(0);
    wave_products<T, ITEMS>(ci, val, x, k0, nk, sp);
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (l + q * kWave <= nr) srp[l + q * kWave] = rpv[q];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = l + q * kWave;
        if (i < nr) {
            const int s = srp[i], e = srp[i + 1];
            double a0 = 0.0, a1 = 0.0;
            int k = s;
            for (; k + 1 < e; k += 2) {
                a0 += sp[k];
                a1 += sp[k + 1];
            }
            if (k < e) a0 += sp[k];
            const T yt = (T)(a0 + a1);
            __builtin_nontemporal_store(yt, y + r0 + i);
            if (w) __builtin_nontemporal_store(fma_t(alpha, yt, xo[q]), w + r0 + i);
        }
    }
    wave_lds_sync();
}

// G lanes per row over rows [r0, r1), one wavefront (64/G rows per pass).
template <typename T, int G>
__device__ __forceinline__ void wave_group_rows(const int32_t *rp, const int32_t *ci, const T *val, const T *x, T *y,
                                                T *w, T alpha, int r0, int r1)
{
    constexpr int RPI = kWave / G;
    const int l = threadIdx.x & (kWave - 1);
    const int lane = l & (G - 1);
    for (int rb = r0; rb < r1; rb += RPI) {
        const int row = rb + l / G;
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
        const double sum = group_sum<G>(a0 + a1);
        if (lane == 0 && row < r1) {
            const T yt = (T)sum;
            y[row] = yt;
            if (w) w[row] = fma_t(alpha, yt, x[row]);
        }
    }
}

}  // namespace spk
