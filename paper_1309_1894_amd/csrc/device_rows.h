// device_rows.h -- per-row work of wavefront tiles, shared by the
// single-matrix row-block kernel and the batched tile kernel.  The row
// stream (short rows' products staged in on-chip memory, then summed per
// row) is the CSR-Stream idea of Greathouse and Daga's CSR-Adaptive
// (SC 2014), applied per wavefront.
#pragma once

#include "device_common.h"

namespace spk {

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

typedef int int4v __attribute__((ext_vector_type(4)));

// Global-address-space views.  Arrays reached through an argument block
// held in memory (a tile record, say) reach the kernel as generic
// pointers, and loads through them compile to flat accesses, which the
// compiler can only wait for all together (vmcnt and lgkmcnt both to
// zero).  Loads through these views are global accesses counted by vmcnt
// alone, so a wait covers just the loads issued before the one needed.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
using gptr_mut = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) { return (gptr<T>)p; }
template <typename T>
__device__ __forceinline__ gptr_mut<T> as_global_mut(T *p) { return (gptr_mut<T>)p; }

// One wavefront streams a run of short rows [r0, r1) with entries [k0, k1)
// (k1 - k0 <= 64*ITEMS, 1 <= r1 - r0 <= 128) through its private LDS slice
// sp (64*ITEMS doubles).  No workgroup barrier: every wavefront of a CU is
// an independent stream.
//
// Loads are issued in the order their data is needed and without
// branches: the column indices first, in 16-byte groups aligned on their
// address (a quarter of the load instructions), then the values (lane l
// takes entries k0 + l + 64j: coalesced 8-byte loads), then the row offsets
// and the rows' own x entries.  Only the index loads are waited for before
// they are staged through the not-yet-used product slice and read back in
// entry order, so the x gathers go out while the values are still
// arriving.  Lanes past the tile's end load the tile's last entry or group
// again (an address in the same page as a valid entry, already cached) and
// drop it.  Then products to LDS and one lane per row sums them (four
// interleaved partial sums).
// With DOT, also returns the lane's part of sum_i x_i*y_i over the tile's
// rows (square matrices: x_i is the row's own entry of x).
// With XW > 0 and xn > 0, the tile's window of x (columns [xlo, xlo + xn),
// xn <= XW, every column of the tile inside it) is copied to the
// wavefront's LDS slice xs with coalesced loads issued together with the
// entry loads (they do not wait for the column indices), and the gathers
// read LDS.
// With CB < 4 (compact columns), ci_ points to CB bytes per entry holding
// the entry's column minus xlo: with CB = 1 (needs XW > 0 and
// 0 < xn <= XW <= 256) its place in the window in LDS; with CB = 2 the
// same, or, when the window is not in LDS (xn = 0), the offset from xlo of
// the x entry gathered from memory.  The bytes travel in the same 16-byte
// groups (16/CB entries each instead of four) and through the same LDS
// staging, so an entry costs CB bytes of index traffic instead of 4;
// everything else, the order of the arithmetic included, is as with
// 4-byte columns.
template <typename T, int ITEMS, bool DOT = false, int XW = 0, int CB = 4>
__device__ __forceinline__ double wave_stream(const int32_t *rp_, const int32_t *ci_, const T *val_, const T *x_,
                                              T *y_, T *w_, T alpha, int r0, int r1, int k0, int k1, double *sp,
                                              int *srp, int xlo = 0, int xn = 0, T *xs = nullptr)
{
    static_assert(CB == 4 || CB == 2 || CB == 1, "columns of 4, 2 or 1 bytes");
    static_assert(CB != 1 || (XW > 0 && XW <= 256), "one-byte columns index a window of at most 256 entries");
    constexpr int IB = CB;                    // bytes per stored column
    constexpr int GE = 16 / IB;               // entries per 16-byte group
    constexpr int STEPS = (ITEMS * kWave + GE - 1 + GE * kWave - 1) / (GE * kWave);
    static_assert(STEPS * 16 * kWave <= 8 * kWave * ITEMS, "staged index groups must fit the product slice");
    const gptr<int32_t> rp = as_global(rp_);
    const gptr<uint8_t> cb = as_global(reinterpret_cast<const uint8_t *>(ci_));
    const gptr<T> val = as_global(val_);
    const gptr<T> x = as_global(x_);
    const gptr_mut<T> y = as_global_mut(y_);
    const gptr_mut<T> w = w_ ? as_global_mut(w_) : nullptr;
    const int l = threadIdx.x & (kWave - 1);
    const int nr = r1 - r0;
    const int nk = k1 - k0;
    if (nr <= 0) return 0.0;
    uint8_t *scb = reinterpret_cast<uint8_t *>(sp);   // 8*64*ITEMS bytes of room
    // entries before k0 in the first group
    const int off = (int)(((uintptr_t)ci_ + (uintptr_t)k0 * IB) & 15u) / IB;
    const int klast = nk > 0 ? nk - 1 : 0;
    int4v g[STEPS];
    T v[ITEMS];
    if (nk > 0) {
        const gptr<uint8_t> cg = cb + ((int64_t)k0 - off) * IB;
        const int glast = (off + klast) & ~(GE - 1);   // start of the last group holding an entry
#pragma unroll
        for (int s = 0; s < STEPS; ++s)
            g[s] = __builtin_nontemporal_load((gptr<int4v>)(cg + IB * min(GE * (l + kWave * s), glast)));
        // matrix entries are read exactly once: non-temporal, so the cache
        // keeps the x entries that neighbouring rows share
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) v[j] = __builtin_nontemporal_load(val + k0 + min(l + j * kWave, klast));
    }
    constexpr int XQ = XW > 0 ? XW / kWave : 1;
    T xwv[XQ];
    const bool win = XW > 0 && xn > 0;
    if constexpr (XW > 0) {
        if (win) {
#pragma unroll
            for (int q = 0; q < XQ; ++q) xwv[q] = x[xlo + min(l + q * kWave, xn - 1)];
        }
    }
    int rpv[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) rpv[q] = rp[r0 + min(l + q * kWave, nr)] - k0;
    T xo[2] = {T(0), T(0)};
    if (DOT || w) {
#pragma unroll
        for (int q = 0; q < 2; ++q) xo[q] = x[r0 + min(l + q * kWave, nr - 1)];
    }
    if (nk > 0) {
#pragma unroll
        for (int s = 0; s < STEPS; ++s) *(int4v *)(scb + 16 * (l + kWave * s)) = g[s];
        if constexpr (XW > 0) {
            if (win) {
#pragma unroll
                for (int q = 0; q < XQ; ++q)
                    if (l + q * kWave < xn) xs[l + q * kWave] = xwv[q];
            }
        }
        wave_lds_sync();
        int c[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int q = min(l + j * kWave, klast) + off;
            if constexpr (CB == 1) c[j] = scb[q];
            else if constexpr (CB == 2) c[j] = reinterpret_cast<const uint16_t *>(scb)[q];
            else c[j] = reinterpret_cast<const int *>(scb)[q];
        }
        wave_lds_sync();   // the staged indices are read before products overwrite them
        T xv[ITEMS];
        if constexpr (CB == 1) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) xv[j] = xs[c[j]];
        } else if constexpr (CB == 2) {
            if (win) {
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) xv[j] = xs[c[j]];
            } else {
#pragma unroll
                for (int j = 0; j < ITEMS; ++j) xv[j] = x[xlo + c[j]];
            }
        } else if (win) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) xv[j] = xs[c[j] - xlo];
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) xv[j] = x[c[j]];
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = l + j * kWave;
            if (k < nk) sp[k] = (double)v[j] * (double)xv[j];
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (l + q * kWave <= nr) srp[l + q * kWave] = rpv[q];
    wave_lds_sync();
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = l + q * kWave;
        if (i < nr) {
            // four interleaved partial sums: four LDS reads in flight
            const int s = srp[i], e = srp[i + 1];
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int k = s;
            for (; k + 3 < e; k += 4) {
                a0 += sp[k];
                a1 += sp[k + 1];
                a2 += sp[k + 2];
                a3 += sp[k + 3];
            }
            if (k < e) a0 += sp[k];
            if (k + 1 < e) a1 += sp[k + 1];
            if (k + 2 < e) a2 += sp[k + 2];
            const T yt = (T)((a0 + a1) + (a2 + a3));
            __builtin_nontemporal_store(yt, y + r0 + i);
            if (w) __builtin_nontemporal_store(fma_t(alpha, yt, xo[q]), w + r0 + i);
            if constexpr (DOT) dot = fma_t((double)xo[q], (double)yt, dot);
        }
    }
    wave_lds_sync();
    return dot;
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

// Rows [r0, r1) one after another, each with all 64 lanes of one
// wavefront: per pass every lane issues UNR value/column loads, then UNR x
// gathers, before it accumulates, so a row keeps 64*UNR gathers in flight
// (the gathers of random-column rows are latency-bound).  UNR partial sums
// per lane, combined in a fixed order, then the wavefront sum.
template <typename T, int UNR, bool DOT = false>
__device__ __forceinline__ double wave_rows_mlp(const int32_t *rp, const int32_t *ci, const T *val, const T *x, T *y,
                                                T *w, T alpha, int r0, int r1)
{
    const int l = threadIdx.x & (kWave - 1);
    double dot = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int s = rp[row], e = rp[row + 1];
        double acc[UNR];
#pragma unroll
        for (int j = 0; j < UNR; ++j) acc[j] = 0.0;
        for (int base = s; base < e; base += kWave * UNR) {
            T v[UNR];
            int c[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int k = base + l + j * kWave;
                v[j] = k < e ? __builtin_nontemporal_load(val + k) : T(0);
                c[j] = k < e ? __builtin_nontemporal_load(ci + k) : -1;
            }
            T xv[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j) xv[j] = c[j] >= 0 ? x[c[j]] : T(0);
#pragma unroll
            for (int j = 0; j < UNR; ++j) acc[j] = fma_t((double)v[j], (double)xv[j], acc[j]);
        }
#pragma unroll
        for (int d = 1; d < UNR; d *= 2)
#pragma unroll
            for (int j = 0; j + d < UNR; j += 2 * d) acc[j] += acc[j + d];
        const double sum = group_sum<kWave>(acc[0]);
        if (l == 0) {
            const T yt = (T)sum;
            y[row] = yt;
            if (w) w[row] = fma_t(alpha, yt, x[row]);
            if constexpr (DOT) dot = fma_t((double)x[row], (double)yt, dot);
        }
    }
    return dot;
}

}  // namespace spk
