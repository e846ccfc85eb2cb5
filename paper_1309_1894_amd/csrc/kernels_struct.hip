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
#include "kernels.h"

namespace spk {

// Both kernels issue all of a row's loads before any product: an absent
// entry's load goes to a clamped in-bounds address and its product is
// dropped by a select (never multiplied by zero, so Inf/NaN in x do not
// leak), so no load waits behind a branch.  Row blocks are remapped so
// each XCD walks a contiguous range of rows and neighbouring rows' x
// entries meet in its L2.

// One lane per row.  The offsets live in the kernel arguments; the loop over
// the kMaxDiag slots is unrolled so they are indexed statically.
template <typename T, int BS, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_dia(DiaArgs a)
{
    const int i = xcd_remap((int)blockIdx.x, (int)gridDim.x) * BS + (int)threadIdx.x;
    if (i >= a.m) return;
    const T *val = (const T *)a.val;
    const T *x = (const T *)a.x;
    const uint32_t msk = a.mask[i];
    T v[kMaxDiag], xv[kMaxDiag];
#pragma unroll
    for (int d = 0; d < kMaxDiag; ++d) {
        if (d < a.ndiag) {
            const int c = min(max(i + a.off[d], 0), a.ncols - 1);
            v[d] = val[(int64_t)d * a.m + i];
            xv[d] = x[c];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < kMaxDiag; ++d) {
        if (d < a.ndiag) {
            const double t = fma_t((double)v[d], (double)xv[d], acc);
            acc = ((msk >> d) & 1u) ? t : acc;
        }
    }
    const T yt = (T)acc;
    ((T *)a.y)[i] = yt;
    if constexpr (FUSED) ((T *)a.w)[i] = fma_t((T)a.alpha, yt, x[i]);
}

// One lane per row of the grid; the neighbours in ascending offset order.
template <typename T, int BS, int DIM, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_stencil(StencilArgs a)
{
    const int r = xcd_remap((int)blockIdx.x, (int)gridDim.x) * BS + (int)threadIdx.x;
    if (r >= a.n) return;
    const T *x = (const T *)a.x;
    const uint32_t ur = (uint32_t)r;
    const uint32_t N3 = (uint32_t)a.N3, N2 = (uint32_t)a.N2;
    const uint32_t k = ur % N3;
    const uint32_t pencil = ur / N3;
    const uint32_t j = DIM >= 2 ? pencil % N2 : 0u;
    const uint32_t i = DIM >= 3 ? pencil / N2 : 0u;
    const int plane = a.N2 * a.N3;
    const int last = a.n - 1;
    const bool has[7] = {DIM >= 3 && i > 0, DIM >= 2 && j > 0, k > 0, true, k + 1 < N3,
                         DIM >= 2 && j + 1 < N2, DIM >= 3 && i + 1 < (uint32_t)a.N1};
    const int at[7] = {max(r - plane, 0), max(r - a.N3, 0), max(r - 1, 0), r,
                       min(r + 1, last), min(r + a.N3, last), min(r + plane, last)};
    T xv[7];
#pragma unroll
    for (int q = 0; q < 7; ++q)
        if ((q == 0 || q == 6) ? DIM >= 3 : (q == 1 || q == 5) ? DIM >= 2 : true) xv[q] = x[at[q]];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        if ((q == 0 || q == 6) ? DIM >= 3 : (q == 1 || q == 5) ? DIM >= 2 : true) {
            const double t = fma_t(a.coef[q], (double)xv[q], acc);
            acc = has[q] ? t : acc;
        }
    }
    const T yt = (T)acc;
    ((T *)a.y)[r] = yt;
    if constexpr (FUSED) ((T *)a.w)[r] = fma_t((T)a.alpha, yt, xv[3]);
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

template <typename T, int BS, bool F>
hipError_t L_dia(const void *p, hipStream_t s)
{
    const DiaArgs &a = *(const DiaArgs *)p;
    hipLaunchKernelGGL((k_spmv_dia<T, BS, F>), dim3((unsigned)((a.m + BS - 1) / BS)), dim3(BS), 0, s, a);
    return hipGetLastError();
}

template <typename T, int BS, bool F>
hipError_t L_stencil(const void *p, hipStream_t s)
{
    const StencilArgs &a = *(const StencilArgs *)p;
    const dim3 g((unsigned)((a.n + BS - 1) / BS));
    if (a.dim == 3)
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 3, F>), g, dim3(BS), 0, s, a);
    else if (a.dim == 2)
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 2, F>), g, dim3(BS), 0, s, a);
    else
        hipLaunchKernelGGL((k_spmv_stencil<T, BS, 1, F>), g, dim3(BS), 0, s, a);
    return hipGetLastError();
}

#define SFN4(L, BS) {{L<float, BS, false>, L<float, BS, true>}, {L<double, BS, false>, L<double, BS, true>}}

const StructEntry kStruct[] = {
    {5, 128, SFN4(L_dia, 128)},     {5, 256, SFN4(L_dia, 256)},     {5, 512, SFN4(L_dia, 512)},
    {6, 128, SFN4(L_stencil, 128)}, {6, 256, SFN4(L_stencil, 256)}, {6, 512, SFN4(L_stencil, 512)},
};

#undef SFN4

}  // namespace

const StructEntry *struct_table(int *count)
{
    *count = (int)(sizeof(kStruct) / sizeof(kStruct[0]));
    return kStruct;
}

}  // namespace spk
