// kernels_struct.hip -- SpMV in structured formats for gfx950.
//
// For matrices whose nonzeros sit on a few diagonals (banded, grid
// operators) the column indices are implied by the diagonal offsets, and
// for a constant-coefficient grid stencil the values are too.  Dropping them
// cuts the bytes an HBM-bound SpMV has to move: on the 7-point Laplacian,
// CSR moves 12 bytes per entry (value + column) plus the row pointers; DIA
// moves 8 bytes per (diagonal, row) plus a 2-byte mask per row; the stencil
// moves only x and y.  Both kernels add a row's products in ascending
// column order with fused multiply-adds, i.e. in the storage order of a CSR
// row with sorted columns, and skip absent entries (an absent entry is not
// a stored zero: 0 * Inf would be NaN).
#include "device_common.h"
#include "device_stencil.h"
#include "kernels.h"

namespace spk {

// Both kernels issue all of a row's loads before any product: an absent
// entry's load goes to a clamped in-bounds address and its product is
// dropped by a select (never multiplied by zero, so Inf/NaN in x do not
// leak), so no load waits behind a branch.  A lane takes ROWS rows (BS
// apart, so every access stays coalesced) to keep enough bytes in flight:
// with one row per lane the stencil moves only 16 bytes per lane and is
// latency-bound.  Row blocks are remapped so each XCD walks a contiguous
// range of rows and neighbouring rows' x entries meet in its L2.

template <typename T, int BS, int ROWS, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_dia(DiaArgs a)
{
    const int base = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (BS * ROWS) + (int)threadIdx.x;
    const T *val = (const T *)a.val;
    const T *x = (const T *)a.x;
    uint32_t msk[ROWS];
    T v[ROWS][kMaxDiag], xv[ROWS][kMaxDiag];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = min(base + u * BS, a.m - 1);
        msk[u] = base + u * BS < a.m ? a.mask[i] : 0u;
#pragma unroll
        for (int d = 0; d < kMaxDiag; ++d) {
            if (d < a.ndiag) {
                const int c = min(max(i + a.off[d], 0), a.ncols - 1);
                v[u][d] = val[(int64_t)d * a.m + i];
                xv[u][d] = x[c];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = base + u * BS;
        if (i >= a.m) break;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < kMaxDiag; ++d) {
            if (d < a.ndiag) {
                const double t = fma_t((double)v[u][d], (double)xv[u][d], acc);
                acc = ((msk[u] >> d) & 1u) ? t : acc;
            }
        }
        const T yt = (T)acc;
        ((T *)a.y)[i] = yt;
        if constexpr (FUSED) ((T *)a.w)[i] = fma_t((T)a.alpha, yt, x[i]);
    }
}

template <typename T, int BS, int DIM, int ROWS, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_stencil(StencilArgs a)
{
    const int base = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (BS * ROWS) + (int)threadIdx.x;
    const T *x = (const T *)a.x;
    T xv[ROWS][7];
    bool has[ROWS][7];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        int at[7];
        stencil_row<DIM>(a, min(base + u * BS, a.n - 1), at, has[u]);
#pragma unroll
        for (int q = 0; q < 7; ++q)
            if (stencil_slot<DIM>(q)) xv[u][q] = x[at[q]];
    }
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int r = base + u * BS;
        if (r >= a.n) break;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            if (stencil_slot<DIM>(q)) {
                const double t = fma_t(a.coef[q], (double)xv[u][q], acc);
                acc = has[u][q] ? t : acc;
            }
        }
        const T yt = (T)acc;
        ((T *)a.y)[r] = yt;
        if constexpr (FUSED) ((T *)a.w)[r] = fma_t((T)a.alpha, yt, xv[u][3]);
    }
}

// The stencil with x staged through LDS: a workgroup copies the x values of
// its rows and one grid line of halo on each side into LDS with coalesced
// loads, then every in-plane neighbour (+-1, +-N3) comes from LDS and only
// the two plane neighbours (+-N2*N3) from global memory: about three global
// loads per row instead of seven.  Same products, same order as
// k_spmv_stencil, so the same bits.
template <typename T, int BS, int DIM, int ROWS, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_stencil_lds(StencilArgs a)
{
    extern __shared__ unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    constexpr int SPAN = BS * ROWS;
    const T *x = (const T *)a.x;
    const int halo = DIM >= 2 ? a.N3 : 1;
    const int R0 = xcd_remap((int)blockIdx.x, (int)gridDim.x) * SPAN;
    const int lo = R0 - halo;
    const int cnt = SPAN + 2 * halo;
    for (int t = (int)threadIdx.x; t < cnt; t += BS) {
        const int g = lo + t;
        xs[t] = (g >= 0 && g < a.n) ? x[g] : T(0);
    }
    const int last = a.n - 1;
    T xp[ROWS][2];
    bool has[ROWS][7];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        int at[7];
        stencil_row<DIM>(a, min(R0 + u * BS + (int)threadIdx.x, last), at, has[u]);
        if constexpr (DIM >= 3) {
            xp[u][0] = x[at[0]];
            xp[u][1] = x[at[6]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int r = R0 + u * BS + (int)threadIdx.x;
        if (r >= a.n) break;
        const int o = r - lo;
        double acc = 0.0;
        double t;
        if constexpr (DIM >= 3) {
            t = fma_t(a.coef[0], (double)xp[u][0], acc);
            acc = has[u][0] ? t : acc;
        }
        if constexpr (DIM >= 2) {
            t = fma_t(a.coef[1], (double)xs[o - a.N3], acc);
            acc = has[u][1] ? t : acc;
        }
        t = fma_t(a.coef[2], (double)xs[o - 1], acc);
        acc = has[u][2] ? t : acc;
        const T xr = xs[o];
        acc = fma_t(a.coef[3], (double)xr, acc);
        t = fma_t(a.coef[4], (double)xs[o + 1], acc);
        acc = has[u][4] ? t : acc;
        if constexpr (DIM >= 2) {
            t = fma_t(a.coef[5], (double)xs[o + a.N3], acc);
            acc = has[u][5] ? t : acc;
        }
        if constexpr (DIM >= 3) {
            t = fma_t(a.coef[6], (double)xp[u][1], acc);
            acc = has[u][6] ? t : acc;
        }
        const T yt = (T)acc;
        ((T *)a.y)[r] = yt;
        if constexpr (FUSED) ((T *)a.w)[r] = fma_t((T)a.alpha, yt, xr);
    }
}

// CSR -> DIA, one lane per row.
template <typename T>
__global__ __launch_bounds__(256) void k_csr_to_dia(int32_t m, const int32_t *rp, const int32_t *ci, const T *val,
                                                    DiaArgs d, T *val_dia, uint16_t *mask)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= m) return;
    uint32_t msk = 0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int o = ci[k] - i;
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q) {
            if (q < d.ndiag && d.off[q] == o) {
                val_dia[(int64_t)q * m + i] = val[k];
                msk |= 1u << q;
            }
        }
    }
    mask[i] = (uint16_t)msk;
}

hipError_t launch_csr_to_dia(int dtype, int32_t m, const int32_t *rp, const int32_t *ci, const void *val,
                             int32_t ndiag, const int32_t *off_host, void *val_dia, uint16_t *mask, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    DiaArgs d{};
    d.ndiag = ndiag;
    for (int q = 0; q < ndiag && q < kMaxDiag; ++q) d.off[q] = off_host[q];
    const dim3 g((unsigned)((m + 255) / 256));
    if (dtype == 1)
        hipLaunchKernelGGL(k_csr_to_dia<double>, g, dim3(256), 0, s, m, rp, ci, (const double *)val, d,
                           (double *)val_dia, mask);
    else
        hipLaunchKernelGGL(k_csr_to_dia<float>, g, dim3(256), 0, s, m, rp, ci, (const float *)val, d,
                           (float *)val_dia, mask);
    return hipGetLastError();
}

namespace {

template <typename T, int BS, int ROWS, bool F>
hipError_t L_dia(const void *p, hipStream_t s)
{
    const DiaArgs &a = *(const DiaArgs *)p;
    const int per = BS * ROWS;
    hipLaunchKernelGGL((k_spmv_dia<T, BS, ROWS, F>), dim3((unsigned)((a.m + per - 1) / per)), dim3(BS), 0, s, a);
    return hipGetLastError();
}

template <typename T, int BS, int ROWS, bool F>
hipError_t L_stencil(const void *p, hipStream_t s)
{
    const StencilArgs &a = *(const StencilArgs *)p;
    const int per = BS * ROWS;
    const dim3 g((unsigned)((a.n + per - 1) / per));
    if (a.dim == 3)
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 3, ROWS, F>), g, dim3(BS), 0, s, a);
    else if (a.dim == 2)
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 2, ROWS, F>), g, dim3(BS), 0, s, a);
    else
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 1, ROWS, F>), g, dim3(BS), 0, s, a);
    return hipGetLastError();
}

template <typename T, int BS, int ROWS, bool F>
hipError_t L_stencil_lds(const void *p, hipStream_t s)
{
    const StencilArgs &a = *(const StencilArgs *)p;
    const int per = BS * ROWS;
    const dim3 g((unsigned)((a.n + per - 1) / per));
    const size_t sh = (size_t)stencil_lds_bytes(BS, ROWS, a.dim, a.N3, (int)sizeof(T));
    if (a.dim == 3)
        hipLaunchKernelGGL((k_spmv_stencil_lds<T, BS, 3, ROWS, F>), g, dim3(BS), sh, s, a);
    else if (a.dim == 2)
        hipLaunchKernelGGL((k_spmv_stencil_lds<T, BS, 2, ROWS, F>), g, dim3(BS), sh, s, a);
    else
        hipLaunchKernelGGL((k_spmv_stencil_lds<T, BS, 1, ROWS, F>), g, dim3(BS), sh, s, a);
    return hipGetLastError();
}

// format, block, rows per lane (the `unroll` knob), LDS staging
#define SFN4(L, BS, R) {{L<float, BS, R, false>, L<float, BS, R, true>}, {L<double, BS, R, false>, L<double, BS, R, true>}}
#define DIA_E(BS, R) {5, BS, R, 0, SFN4(L_dia, BS, R)}
#define STN_E(BS, R) {6, BS, R, 0, SFN4(L_stencil, BS, R)}
#define STL_E(BS, R) {6, BS, R, 1, SFN4(L_stencil_lds, BS, R)}

const StructEntry kStruct[] = {
    DIA_E(128, 1), DIA_E(128, 2), DIA_E(256, 1), DIA_E(256, 2), DIA_E(512, 1), DIA_E(512, 2),
    STN_E(128, 1), STN_E(128, 2), STN_E(128, 4), STN_E(128, 8),
    STN_E(256, 1), STN_E(256, 2), STN_E(256, 4), STN_E(256, 8),
    STN_E(512, 1), STN_E(512, 2), STN_E(512, 4),
    STL_E(256, 2), STL_E(256, 4), STL_E(512, 2), STL_E(512, 4),
};

#undef STL_E
#undef STN_E
#undef DIA_E
#undef SFN4

}  // namespace

const StructEntry *struct_table(int *count)
{
    *count = (int)(sizeof(kStruct) / sizeof(kStruct[0]));
    return kStruct;
}

}  // namespace spk
