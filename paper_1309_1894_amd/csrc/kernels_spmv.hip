// kernels_spmv.hip -- CSR sparse matrix-vector product y = A*x for gfx950,
// optionally fused with the step w = alpha*y + x.
//
// Four kernel families (the code variants the tuner searches):
//   SCALAR   one lane per row: each lane walks its own row.
//   VECTOR   G lanes per row (G = 2..64; 64 is one wavefront per row): the
//            lanes of a group stride the row with coalesced loads and meet
//            in a DPP/ds_swizzle group reduction.  Optionally stages the
//            workgroup's row_ptr slice in LDS.
//   SELL     sliced ELL: slices of C rows stored column-major, one lane per
//            row, fully coalesced, no reduction; rows keep their own length
//            so padding is never read.
//   ADAPTIVE precomputed wavefront tiles: runs of short rows whose entries
//            fit a wavefront's LDS slice are streamed into LDS with
//            coalesced loads and summed per row from LDS; runs of medium
//            rows, and single long rows, get a wavefront (64 lanes per row,
//            eight loads and gathers in flight per lane).  Streaming short
//            rows through on-chip memory and giving long rows a vector of
//            their own is the CSR-Stream / CSR-Adaptive scheme published by
//            Greathouse and Daga (SC 2014); here each wavefront streams its
//            own tile, with no workgroup barrier.
// Products are formed and accumulated in FP64 (FP32 operands are widened
// first, so their products are exact) and each output is rounded once.
#include "device_common.h"
#include "device_rows.h"
#include "kernels.h"

namespace spk {

template <typename T, bool FUSED>
__device__ __forceinline__ void store_row(const SpmvArgs<T> &a, int row, double acc)
{
    const T yt = (T)acc;
    a.y[row] = yt;
    if constexpr (FUSED) a.w[row] = fma_t(a.alpha, yt, a.x[row]);
}

// --------------------------------------------------------------- SCALAR --

// VEC > 1: the row's entries from the first index that is a multiple of
// VEC on are read VEC at a time (one VEC*sizeof(T)-byte value access and one
// VEC*4-byte index access), the few before it and after the last full
// group one at a time; partial sum u takes the u-th entry of each group.
template <typename T, int BS, int UNR, int VEC, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_scalar(SpmvArgs<T> a)
{
    const int row = a.row0 + (int)blockIdx.x * BS + (int)threadIdx.x;
    if (row >= a.row0 + a.m) return;
    const int s = a.rp[row], e = a.rp[row + 1];
    if constexpr (VEC == 1) {
        double acc[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) acc[u] = 0.0;
        int k = s;
        for (; k + UNR <= e; k += UNR) {
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                acc[u] = fma_t((double)a.val[k + u], (double)a.x[a.ci[k + u]], acc[u]);
        }
        for (; k < e; ++k) acc[0] = fma_t((double)a.val[k], (double)a.x[a.ci[k]], acc[0]);
        double sum = acc[0];
#pragma unroll
        for (int u = 1; u < UNR; ++u) sum += acc[u];
        store_row<T, FUSED>(a, row, sum);
    } else {
        double acc[VEC];
#pragma unroll
        for (int u = 0; u < VEC; ++u) acc[u] = 0.0;
        int k = s;
        const int ka = min(e, (s + VEC - 1) / VEC * VEC);
        for (; k < ka; ++k) acc[0] = fma_t((double)a.val[k], (double)a.x[a.ci[k]], acc[0]);
        using VT = vec_t<T, VEC>;
        using VI = vec_t<int32_t, VEC>;
        for (; k + VEC <= e; k += VEC) {
            const VT v = *reinterpret_cast<const VT *>(a.val + k);
            const VI c = *reinterpret_cast<const VI *>(a.ci + k);
#pragma unroll
            for (int u = 0; u < VEC; ++u) acc[u] = fma_t((double)v.v[u], (double)a.x[c.v[u]], acc[u]);
        }
        for (; k < e; ++k) acc[0] = fma_t((double)a.val[k], (double)a.x[a.ci[k]], acc[0]);
        double sum = acc[0];
#pragma unroll
        for (int u = 1; u < VEC; ++u) sum += acc[u];
        store_row<T, FUSED>(a, row, sum);
    }
}

// --------------------------------------------------------------- VECTOR --

// VEC > 1: lanes take groups of VEC consecutive entries (one
// VEC*sizeof(T)-byte value access and one VEC*4-byte index access each),
// from the row's first index that is a multiple of VEC; the entries before
// it and after its last full group go one per lane.
template <typename T, int BS, int G, int UNR, bool LDSRP, int VEC, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_vector(SpmvArgs<T> a)
{
    constexpr int RPB = BS / G;  // rows per workgroup
    const int t = threadIdx.x;
    const int lane = t & (G - 1);
    const int rbase = a.row0 + (int)blockIdx.x * RPB;
    const int rend = a.row0 + a.m;
    const int row = rbase + t / G;
    int s = 0, e = 0;
    if constexpr (LDSRP) {
        __shared__ int srp[RPB + 1];
        for (int i = t; i <= RPB; i += BS) srp[i] = a.rp[min(rbase + i, rend)];
        __syncthreads();
        s = srp[t / G];
        e = srp[t / G + 1];
    } else if (row < rend) {
        s = a.rp[row];
        e = a.rp[row + 1];
    }
    double acc[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) acc[u] = 0.0;
    if constexpr (VEC == 1) {
        for (int k = s + lane; k < e; k += G * UNR) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int kk = k + u * G;
                if (kk < e) acc[u] = fma_t((double)a.val[kk], (double)a.x[a.ci[kk]], acc[u]);
            }
        }
    } else {
        static_assert(G >= 2 * (VEC - 1), "the head and tail entries need a lane each");
        const int ka = min(e, (s + VEC - 1) / VEC * VEC);         // first group boundary
        const int kb = ka + (e - ka) / VEC * VEC;                  // end of the full groups
        // head and tail: at most 2*(VEC-1) entries, one per lane
        {
            const int h = ka - s;
            const int k = lane < h ? s + lane : kb + (lane - h);
            if (lane < h + (e - kb)) acc[0] = fma_t((double)a.val[k], (double)a.x[a.ci[k]], acc[0]);
        }
        using VT = vec_t<T, VEC>;
        using VI = vec_t<int32_t, VEC>;
        for (int k = ka + lane * VEC; k < kb; k += G * VEC) {
            const VT v = *reinterpret_cast<const VT *>(a.val + k);
            const VI c = *reinterpret_cast<const VI *>(a.ci + k);
#pragma unroll
            for (int u = 0; u < VEC; ++u) acc[u % UNR] = fma_t((double)v.v[u], (double)a.x[c.v[u]], acc[u % UNR]);
        }
    }
    double sum = acc[0];
#pragma unroll
    for (int u = 1; u < UNR; ++u) sum += acc[u];
    sum = group_sum<G>(sum);  // every lane of the wavefront takes part
    if (lane == 0 && row < rend) store_row<T, FUSED>(a, row, sum);
}

// ----------------------------------------------------------------- SELL --

template <typename T, int BS, int C, int UNR, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_sell(SpmvArgs<T> a)
{
    const int row = a.row0 + (int)blockIdx.x * BS + (int)threadIdx.x;
    if (row >= a.row0 + a.m) return;
    const int slice = row / C;
    const int64_t base = a.sell_ptr[slice] + (row - slice * C);
    const int len = a.sell_len[row];
    double acc[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) acc[u] = 0.0;
    int k = 0;
    for (; k + UNR <= len; k += UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t p = base + (int64_t)(k + u) * C;
            acc[u] = fma_t((double)a.sell_val[p], (double)a.x[a.sell_ci[p]], acc[u]);
        }
    }
    for (; k < len; ++k) {
        const int64_t p = base + (int64_t)k * C;
        acc[0] = fma_t((double)a.sell_val[p], (double)a.x[a.sell_ci[p]], acc[0]);
    }
    double sum = acc[0];
#pragma unroll
    for (int u = 1; u < UNR; ++u) sum += acc[u];
    store_row<T, FUSED>(a, row, sum);
}

// ------------------------------------------------------------- ADAPTIVE --

// Row blocks are wavefront tiles (precomputed at registration for a
// wavefront capacity of E entries): each wavefront of a workgroup runs its
// own block with a private LDS slice, without workgroup barriers.
// With XW > 0, row-stream blocks whose x window fits XW entries take x from
// LDS (the window copied there beside the entry loads).  With CB = 2,
// row-stream blocks whose columns span at most 65,536 read two-byte column
// offsets from the block's first column (which is also its window's first
// column) instead of the CSR's four-byte columns; the other blocks read
// the CSR's.
template <typename T, int BS, int E, int XW, int CB, bool FUSED>
__global__ __launch_bounds__(BS) void k_spmv_adaptive(SpmvArgs<T> a)
{
    constexpr int NW = BS / kWave;
    __shared__ double sp[NW * E];
    __shared__ int srp[NW * (kWaveTileRows + 1)];
    __shared__ T xs[NW * (XW > 0 ? XW : 1)];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int ngroups = (a.nblk + NW - 1) / NW;
    const int g = xcd_remap((int)blockIdx.x, ngroups);
    const int bl = g * NW + wv;
    if (bl >= a.nblk) return;
    const int b = a.blk0 + bl;
    const uint32_t e0 = a.blocks[b], e1 = a.blocks[b + 1];
    const int r0 = (int)(e0 & kBlkRowMask), r1 = (int)(e1 & kBlkRowMask);
    const uint32_t mode = e0 >> 30;
    T *w = FUSED ? a.w : nullptr;
    if (mode == kBlkStream) {
        int xlo = 0, xn = 0;
        if constexpr (XW > 0) {
            xlo = a.block_x[2 * b];
            xn = a.block_x[2 * b + 1];
            xn = xn <= XW ? xn : 0;
        }
        if constexpr (CB == 2) {
            const int base = a.block_c16[b];
            if (base >= 0) {
                wave_stream<T, E / kWave, false, XW, 2>(a.rp, reinterpret_cast<const int32_t *>(a.c16), a.val, a.x,
                                                        a.y, w, a.alpha, r0, r1, a.block_k[b], a.block_k[b + 1],
                                                        sp + wv * E, srp + wv * (kWaveTileRows + 1), base, xn,
                                                        xs + wv * (XW > 0 ? XW : 1));
                return;
            }
        }
        wave_stream<T, E / kWave, false, XW>(a.rp, a.ci, a.val, a.x, a.y, w, a.alpha, r0, r1, a.block_k[b],
                                             a.block_k[b + 1], sp + wv * E, srp + wv * (kWaveTileRows + 1), xlo, xn,
                                             xs + wv * (XW > 0 ? XW : 1));
    } else {
        // medium rows (kBlkWave) and single long rows (kBlkLong)
        wave_rows_mlp<T, 8>(a.rp, a.ci, a.val, a.x, a.y, w, a.alpha, r0, r1);
    }
}

// --------------------------------------------------- block x windows --

__global__ __launch_bounds__(256) void k_block_windows(const uint32_t *blocks, const int32_t *block_k,
                                                       const int32_t *ci, int32_t nblk, int cap, int32_t *bx)
{
    const int b = (int)blockIdx.x * 4 + (int)threadIdx.x / kWave;
    if (b >= nblk) return;
    const int l = threadIdx.x & (kWave - 1);
    const int k0 = block_k[b], k1 = block_k[b + 1];
    int lo = INT32_MAX, hi = -1;
    if ((blocks[b] >> 30) == kBlkStream)
        for (int k = k0 + l; k < k1; k += kWave) {
            const int c = ci[k];
            lo = min(lo, c);
            hi = max(hi, c);
        }
#pragma unroll
    for (int d = 1; d < kWave; d *= 2) {
        lo = min(lo, __shfl_xor(lo, d));
        hi = max(hi, __shfl_xor(hi, d));
    }
    if (l == 0) {
        const bool fits = hi >= lo && (int64_t)hi - lo + 1 <= cap;
        bx[2 * b] = fits ? lo : 0;
        bx[2 * b + 1] = fits ? hi - lo + 1 : 0;
    }
}

hipError_t launch_block_windows(const uint32_t *blocks, const int32_t *block_k, const int32_t *ci, int32_t nblk,
                                int cap, int32_t *bx, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_windows, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, blocks, block_k, ci, nblk,
                       cap, bx);
    return hipGetLastError();
}

// Two-byte columns of the row-stream blocks, one wavefront per block: a
// block with entries whose columns span at most 65,536 gets base = its
// smallest column and c16[k] = ci[k] - base for its entries; any other
// block gets base = -1 (and keeps reading the CSR's columns).
__global__ __launch_bounds__(256) void k_block_c16(const uint32_t *blocks, const int32_t *block_k,
                                                   const int32_t *ci, int32_t nblk, uint16_t *c16, int32_t *base)
{
    const int b = (int)blockIdx.x * 4 + (int)threadIdx.x / kWave;
    if (b >= nblk) return;
    const int l = threadIdx.x & (kWave - 1);
    const int k0 = block_k[b], k1 = block_k[b + 1];
    const bool stream = (blocks[b] >> 30) == kBlkStream;
    int lo = INT32_MAX, hi = -1;
    if (stream)
        for (int k = k0 + l; k < k1; k += kWave) {
            const int c = ci[k];
            lo = min(lo, c);
            hi = max(hi, c);
        }
#pragma unroll
    for (int d = 1; d < kWave; d *= 2) {
        lo = min(lo, __shfl_xor(lo, d));
        hi = max(hi, __shfl_xor(hi, d));
    }
    const bool fits = hi >= lo && (int64_t)hi - lo < 65536;
    if (fits)
        for (int k = k0 + l; k < k1; k += kWave) c16[k] = (uint16_t)(ci[k] - lo);
    if (l == 0) base[b] = fits ? lo : -1;
}

hipError_t launch_block_c16(const uint32_t *blocks, const int32_t *block_k, const int32_t *ci, int32_t nblk,
                            uint16_t *c16, int32_t *base, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_c16, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, s, blocks, block_k, ci, nblk, c16,
                       base);
    return hipGetLastError();
}

// ------------------------------------------------------------ registry --

namespace {

template <typename T, int BS, int UNR, int VEC, bool F>
hipError_t L_scalar(const void *p, dim3 g, hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_scalar<T, BS, UNR, VEC, F>), g, dim3(BS), 0, s, *(const SpmvArgs<T> *)p);
    return hipGetLastError();
}

template <typename T, int BS, int G, int UNR, bool LDSRP, int VEC, bool F>
hipError_t L_vector(const void *p, dim3 g, hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_vector<T, BS, G, UNR, LDSRP, VEC, F>), g, dim3(BS), 0, s, *(const SpmvArgs<T> *)p);
    return hipGetLastError();
}

template <typename T, int BS, int C, int UNR, bool F>
hipError_t L_sell(const void *p, dim3 g, hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_sell<T, BS, C, UNR, F>), g, dim3(BS), 0, s, *(const SpmvArgs<T> *)p);
    return hipGetLastError();
}

template <typename T, int BS, int E, int XW, int CB, bool F>
hipError_t L_adaptive(const void *p, dim3 g, hipStream_t s)
{
    hipLaunchKernelGGL((k_spmv_adaptive<T, BS, E, XW, CB, F>), g, dim3(BS), 0, s, *(const SpmvArgs<T> *)p);
    return hipGetLastError();
}

#define FN4(L, ...) {{L<float, __VA_ARGS__, false>, L<float, __VA_ARGS__, true>}, \
                     {L<double, __VA_ARGS__, false>, L<double, __VA_ARGS__, true>}}

// format, block, group, unroll, lds (, entries per access)
#define SCALAR(BS, U) {1, BS, 1, U, 0, FN4(L_scalar, BS, U, 1)}
#define SCALAR_V(BS, V) {1, BS, 1, V, 0, FN4(L_scalar, BS, V, V), V}
#define VECTOR(BS, G, U) {2, BS, G, U, 0, FN4(L_vector, BS, G, U, false, 1)}
#define VECTOR_V(BS, G, U, V) {2, BS, G, U, 0, FN4(L_vector, BS, G, U, false, V), V}
#define VECTOR_LDS(BS, G) {2, BS, G, 1, 1, FN4(L_vector, BS, G, 1, true, 1)}
#define SELL(C, U) {3, 256, C, U, 0, FN4(L_sell, 256, C, U)}
// lds = row-stream entries per wavefront tile; group = LDS room for x per
// wavefront (1 = none)
#define ADAPT(BS, E) {4, BS, 1, 1, E, FN4(L_adaptive, BS, E, 0, 4)}
#define ADAPT_X(BS, E) {4, BS, 256, 1, E, FN4(L_adaptive, BS, E, 256, 4)}
// vec = 2: two-byte columns in the row-stream blocks
#define ADAPT_C16(BS, E) {4, BS, 1, 1, E, FN4(L_adaptive, BS, E, 0, 2), 2}
#define ADAPT_C16_X(BS, E) {4, BS, 256, 1, E, FN4(L_adaptive, BS, E, 256, 2), 2}

#define VECTOR_U(BS, G) VECTOR(BS, G, 1), VECTOR(BS, G, 2), VECTOR(BS, G, 4)
#define VECTOR_G(BS) VECTOR_U(BS, 2), VECTOR_U(BS, 4), VECTOR_U(BS, 8), VECTOR_U(BS, 16), \
                     VECTOR_U(BS, 32), VECTOR_U(BS, 64)

const SpmvEntry kSpmv[] = {
    // plain variants first: thread per row, wavefront per row (256 threads)
    SCALAR(256, 1), VECTOR(256, 64, 1),
    SCALAR(64, 1), SCALAR(128, 1), SCALAR(512, 1),
    SCALAR(64, 2), SCALAR(128, 2), SCALAR(256, 2), SCALAR(512, 2),
    SCALAR(64, 4), SCALAR(128, 4), SCALAR(256, 4), SCALAR(512, 4),
    VECTOR_U(128, 2), VECTOR_U(128, 4), VECTOR_U(128, 8), VECTOR_U(128, 16), VECTOR_U(128, 32), VECTOR_U(128, 64),
    VECTOR_U(256, 2), VECTOR_U(256, 4), VECTOR_U(256, 8), VECTOR_U(256, 16), VECTOR_U(256, 32),
    VECTOR(256, 64, 2), VECTOR(256, 64, 4),
    VECTOR_G(512),
    VECTOR_LDS(256, 2), VECTOR_LDS(256, 4), VECTOR_LDS(256, 8), VECTOR_LDS(256, 16),
    SELL(32, 1), SELL(32, 2), SELL(32, 4),
    SELL(64, 1), SELL(64, 2), SELL(64, 4),
    SELL(128, 1), SELL(128, 2), SELL(128, 4),
    SELL(256, 1), SELL(256, 2), SELL(256, 4),
    ADAPT(128, 256), ADAPT(128, 512), ADAPT(128, 1024),
    ADAPT(256, 256), ADAPT(256, 512), ADAPT(256, 1024),
    ADAPT(512, 256), ADAPT(512, 512), ADAPT(512, 1024),
    ADAPT_X(128, 256), ADAPT_X(256, 256), ADAPT_X(256, 512), ADAPT_X(512, 256),
    // one-wavefront workgroups
    ADAPT(64, 256), ADAPT(64, 512), ADAPT(64, 1024), ADAPT_X(64, 256), ADAPT_X(64, 512), ADAPT_X(64, 1024),
    // wider accesses: two entries (16 bytes of FP64 values, 8 of FP32) or
    // four (16 bytes of FP32 values) per access
    SCALAR_V(256, 2), SCALAR_V(256, 4),
    VECTOR_V(256, 4, 2, 2), VECTOR_V(256, 8, 2, 2), VECTOR_V(256, 16, 2, 2), VECTOR_V(256, 32, 2, 2),
    VECTOR_V(256, 64, 2, 2), VECTOR_V(256, 8, 4, 4), VECTOR_V(256, 16, 4, 4), VECTOR_V(256, 64, 4, 4),
    // row blocks with two-byte columns
    ADAPT_C16(64, 256), ADAPT_C16(64, 512), ADAPT_C16(64, 1024), ADAPT_C16(128, 256), ADAPT_C16(128, 512),
    ADAPT_C16(256, 256), ADAPT_C16(256, 512), ADAPT_C16(512, 256),
    ADAPT_C16_X(256, 256), ADAPT_C16_X(64, 256),
};

}  // namespace

const SpmvEntry *spmv_table(int *count)
{
    *count = (int)(sizeof(kSpmv) / sizeof(kSpmv[0]));
    return kSpmv;
}

}  // namespace spk
