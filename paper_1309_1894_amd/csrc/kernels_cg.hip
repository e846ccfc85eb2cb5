// kernels_cg.hip -- conjugate-gradient iteration on the library's kernels.
//
// One CG iteration (textbook order) needs q = A p, p.q, two AXPYs, r.r and
// the direction update p = r + beta p.  Composed from separate library calls
// that is one SpMV, two dot passes, three vector passes and two host round
// trips for the step sizes.  Here it is three launches with every scalar
// kept on the device:
//
//   k_cg_spmv_dot   q = A p on the wavefront tiles of the matrix; each
//                   workgroup also leaves its part of p.q (the own-row entry
//                   of p is already loaded for the tile).
//   k_cg_residual   alpha = r.r / p.q from those parts, r -= alpha q and
//                   this workgroup's part of the new r.r.
//   k_cg_direction  beta = r'.r' / r.r from those parts, then x += alpha p
//                   and p = r + beta p in one pass over p (x's update waits
//                   for this pass so that p is read once); the first
//                   workgroup records r'.r'.
//
// A reduction is finished by the kernel that consumes it: every workgroup
// of the consumer adds the producer's partials in the same fixed order, so
// all of them hold the same bits and no workgroup of the producer has to
// publish its partial with a device-scope release (on this GPU such a
// release writes back the XCD's L2 and serialises there, which costs more
// than the whole SpMV at thousands of workgroups).  A step size whose
// denominator is exactly zero is taken as zero.
#include "device_rows.h"
#include "device_stencil.h"
#include "kernels.h"

namespace spk {

typedef double f64x2_t __attribute__((ext_vector_type(2)));

namespace {

// Sum of part[0, n) in a fixed order (lane-strided, then the block tree),
// returned to every thread.
template <int BS>
__device__ __forceinline__ double sum_partials(const double *part, int64_t n, double *red)
{
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BS) a += part[i];
    return block_sum<BS>(a, red);
}

}  // namespace

// q = A p over wavefront tiles: wavefront w of workgroup b runs tile w of
// tile group xcd_remap(b) (runs of neighbouring groups per XCD, so groups in
// flight on an XCD share their x entries in its L2), and the workgroup
// leaves its part of p.q at that group's index.  With CB = 2 the row-stream
// tiles that have two-byte columns read those (offsets from the tile's
// first column) instead of the CSR's.
template <int BS, int E, int CB>
__global__ __launch_bounds__(BS) void k_cg_spmv_dot(CgLaunch c)
{
    constexpr int NW = BS / kWave;
    __shared__ double sp[NW * E];
    __shared__ int srp[NW * (kWaveTileRows + 1)];
    __shared__ double red[NW];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int g = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int bl = g * NW + wv;
    const double *p = c.spmv_x;
    double d = 0.0;
    if (bl < c.nblk) {
        const uint32_t e0 = c.blocks[bl], e1 = c.blocks[bl + 1];
        const int r0 = (int)(e0 & kBlkRowMask), r1 = (int)(e1 & kBlkRowMask);
        const int base = CB == 2 ? c.block_c16[bl] : -1;
        if ((e0 >> 30) == kBlkStream && CB == 2 && base >= 0)
            d = wave_stream<double, E / kWave, true, 0, 2>(c.rp, reinterpret_cast<const int32_t *>(c.c16), c.val,
                                                           p, c.q, nullptr, 0.0, r0, r1, c.block_k[bl],
                                                           c.block_k[bl + 1], sp + wv * E,
                                                           srp + wv * (kWaveTileRows + 1), base, 0);
        else if ((e0 >> 30) == kBlkStream)
            d = wave_stream<double, E / kWave, true>(c.rp, c.ci, c.val, p, c.q, nullptr, 0.0, r0, r1,
                                                     c.block_k[bl], c.block_k[bl + 1], sp + wv * E,
                                                     srp + wv * (kWaveTileRows + 1));
        else
            d = wave_rows_mlp<double, 8, true>(c.rp, c.ci, c.val, p, c.q, nullptr, 0.0, r0, r1);
    }
    if (!c.part1) return;   // same for the whole grid
    d = block_sum<BS>(d, red);
    if (threadIdx.x == 0) c.part1[g] = d;
}

// q = A p for a constant-coefficient grid stencil (no matrix arrays): a
// lane takes ROWS rows BS apart per pass of a grid-stride loop, all their
// loads first (clamped addresses, absent neighbours dropped by a select),
// neighbours added in ascending offset order as in k_spmv_stencil; each
// workgroup leaves its part of p.q.  Workgroups are remapped so each XCD
// sweeps contiguous rows.
template <int BS, int DIM, int ROWS>
__global__ __launch_bounds__(BS) void k_cg_stencil_dot(CgLaunch c)
{
    __shared__ double red[BS / kWave];
    const StencilArgs &a = c.st;
    const double *p = c.spmv_x;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int stride = (int)gridDim.x * BS * ROWS;
    double d = 0.0;
    for (int base = b * BS * ROWS + (int)threadIdx.x; base < a.n; base += stride) {
        double pv[ROWS][7];
        bool has[ROWS][7];
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            int at[7];
            stencil_row<DIM>(a, min(base + u * BS, a.n - 1), at, has[u]);
#pragma unroll
            for (int q = 0; q < 7; ++q)
                if (stencil_slot<DIM>(q)) pv[u][q] = p[at[q]];
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int r = base + u * BS;
            if (r >= a.n) break;
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                if (stencil_slot<DIM>(q)) {
                    const double t = fma_t(a.coef[q], pv[u][q], acc);
                    acc = has[u][q] ? t : acc;
                }
            }
            __builtin_nontemporal_store(acc, c.q + r);
            d = fma_t(pv[u][3], acc, d);
        }
    }
    if (!c.part1) return;   // same for the whole grid
    d = block_sum<BS>(d, red);
    if (threadIdx.x == 0) c.part1[blockIdx.x] = d;
}

// The same with p staged through LDS (as k_spmv_stencil_lds): per pass a
// workgroup copies p of its BS*ROWS rows and one grid line of halo on each
// side into LDS (dynamic shared memory, stencil_lds_bytes), so only the
// plane neighbours come from global memory.  Same products, same order.
template <int BS, int DIM, int ROWS>
__global__ __launch_bounds__(BS) void k_cg_stencil_lds(CgLaunch c)
{
    extern __shared__ double ps[];
    __shared__ double red[BS / kWave];
    constexpr int SPAN = BS * ROWS;
    const StencilArgs &a = c.st;
    const double *p = c.spmv_x;
    const int halo = DIM >= 2 ? a.N3 : 1;
    const int cnt = SPAN + 2 * halo;
    const int last = a.n - 1;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int stride = (int)gridDim.x * SPAN;
    double d = 0.0;
    for (int R0 = b * SPAN; R0 < a.n; R0 += stride) {
        const int lo = R0 - halo;
        __syncthreads();   // the previous pass has finished reading ps
        for (int t = (int)threadIdx.x; t < cnt; t += BS) {
            const int g = lo + t;
            ps[t] = (g >= 0 && g < a.n) ? p[g] : 0.0;
        }
        double pp[ROWS][2];
        bool has[ROWS][7];
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            int at[7];
            stencil_row<DIM>(a, min(R0 + u * BS + (int)threadIdx.x, last), at, has[u]);
            if constexpr (DIM >= 3) {
                pp[u][0] = p[at[0]];
                pp[u][1] = p[at[6]];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int r = R0 + u * BS + (int)threadIdx.x;
            if (r >= a.n) break;
            const int o = r - lo;
            double acc = 0.0, t;
            if constexpr (DIM >= 3) {
                t = fma_t(a.coef[0], pp[u][0], acc);
                acc = has[u][0] ? t : acc;
            }
            if constexpr (DIM >= 2) {
                t = fma_t(a.coef[1], ps[o - a.N3], acc);
                acc = has[u][1] ? t : acc;
            }
            t = fma_t(a.coef[2], ps[o - 1], acc);
            acc = has[u][2] ? t : acc;
            const double pr = ps[o];
            acc = fma_t(a.coef[3], pr, acc);
            t = fma_t(a.coef[4], ps[o + 1], acc);
            acc = has[u][4] ? t : acc;
            if constexpr (DIM >= 2) {
                t = fma_t(a.coef[5], ps[o + a.N3], acc);
                acc = has[u][5] ? t : acc;
            }
            if constexpr (DIM >= 3) {
                t = fma_t(a.coef[6], pp[u][1], acc);
                acc = has[u][6] ? t : acc;
            }
            __builtin_nontemporal_store(acc, c.q + r);
            d = fma_t(pr, acc, d);
        }
    }
    if (!c.part1) return;   // same for the whole grid
    d = block_sum<BS>(d, red);
    if (threadIdx.x == 0) c.part1[blockIdx.x] = d;
}

// alpha = rr / p.q, r -= alpha q, part2 = this workgroup's r.r; the first
// workgroup stores alpha for the direction kernel.  Two doubles per lane
// access, UNR accesses in flight; the first chunk's loads are issued before
// p.q is assembled.
template <int BS, int UNR>
__global__ __launch_bounds__(BS) void k_cg_residual(CgLaunch c)
{
    constexpr int64_t PER = (int64_t)BS * 2 * UNR;
    __shared__ double red[BS / kWave];
    const int t = threadIdx.x;
    const int64_t n = c.n;
    const int64_t stride = (int64_t)gridDim.x * PER;
    int64_t base = (int64_t)blockIdx.x * PER;
    f64x2_t rv[UNR], qv[UNR];
    auto load = [&](int64_t at) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t i = at + ((int64_t)u * BS + t) * 2;
            rv[u] = *(const f64x2_t *)(c.r + i);
            qv[u] = __builtin_nontemporal_load((const f64x2_t *)(c.q + i));
        }
    };
    bool full = base + PER <= n;
    if (full) load(base);
    const double pq = sum_partials<BS>(c.part1, c.spmv_grid, red);
    const double rr = c.sc[c.slot];
    const double alpha = pq != 0.0 ? rr / pq : 0.0;
    if (blockIdx.x == 0 && t == 0) c.sc[kCgAlpha] = alpha;
    double acc[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) acc[u] = 0.0;
    for (; base < n; base += stride) {
        if (full) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t i = base + ((int64_t)u * BS + t) * 2;
                f64x2_t rn;
                rn[0] = fma_t(-alpha, qv[u][0], rv[u][0]);
                rn[1] = fma_t(-alpha, qv[u][1], rv[u][1]);
                acc[u] = fma_t(rn[0], rn[0], acc[u]);
                acc[u] = fma_t(rn[1], rn[1], acc[u]);
                *(f64x2_t *)(c.r + i) = rn;
            }
        } else {
            for (int64_t i = base + t; i < n && i < base + PER; i += BS) {
                const double rn = fma_t(-alpha, c.q[i], c.r[i]);
                c.r[i] = rn;
                acc[0] = fma_t(rn, rn, acc[0]);
            }
        }
        full = base + stride + PER <= n;
        if (full) load(base + stride);
    }
    double s = acc[0];
#pragma unroll
    for (int u = 1; u < UNR; ++u) s += acc[u];
    s = block_sum<BS>(s, red);
    if (t == 0) c.part2[blockIdx.x] = s;
}

// beta = rr' / rr with rr' the sum of part2, then x += alpha p and
// p = r + beta p (both from the same p); the first workgroup records rr'
// (hist, and the other scalar slot).
template <int BS, int UNR>
__global__ __launch_bounds__(BS) void k_cg_direction(CgLaunch c)
{
    constexpr int64_t PER = (int64_t)BS * 2 * UNR;
    __shared__ double red[BS / kWave];
    const int t = threadIdx.x;
    const int64_t n = c.n;
    const int64_t stride = (int64_t)gridDim.x * PER;
    int64_t base = (int64_t)blockIdx.x * PER;
    f64x2_t xv[UNR], rv[UNR], pv[UNR];
    auto load = [&](int64_t at) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t i = at + ((int64_t)u * BS + t) * 2;
            xv[u] = __builtin_nontemporal_load((const f64x2_t *)(c.x + i));
            rv[u] = __builtin_nontemporal_load((const f64x2_t *)(c.r + i));
            pv[u] = *(const f64x2_t *)(c.p + i);
        }
    };
    bool full = base + PER <= n;
    if (full) load(base);
    const double rr_new = sum_partials<BS>(c.part2, c.grid, red);
    const double rr = c.sc[c.slot];
    const double beta = rr != 0.0 ? rr_new / rr : 0.0;
    const double alpha = c.sc[kCgAlpha];
    if (blockIdx.x == 0 && t == 0) {
        c.sc[c.slot ^ 1] = rr_new;
        *c.hist = rr_new;
    }
    for (; base < n; base += stride) {
        if (full) {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t i = base + ((int64_t)u * BS + t) * 2;
                f64x2_t xn, pn;
                xn[0] = fma_t(alpha, pv[u][0], xv[u][0]);
                xn[1] = fma_t(alpha, pv[u][1], xv[u][1]);
                pn[0] = fma_t(beta, pv[u][0], rv[u][0]);
                pn[1] = fma_t(beta, pv[u][1], rv[u][1]);
                __builtin_nontemporal_store(xn, (f64x2_t *)(c.x + i));
                *(f64x2_t *)(c.p + i) = pn;
            }
        } else {
            for (int64_t i = base + t; i < n && i < base + PER; i += BS) {
                const double pi = c.p[i];
                c.x[i] = fma_t(alpha, pi, c.x[i]);
                c.p[i] = fma_t(beta, pi, c.r[i]);
            }
        }
        full = base + stride + PER <= n;
        if (full) load(base + stride);
    }
}

// Start of the solve, after q = A x: r = b - q, p = r, part2 = r.r parts.
template <int BS, int UNR>
__global__ __launch_bounds__(BS) void k_cg_start(CgLaunch c)
{
    constexpr int64_t PER = (int64_t)BS * 2 * UNR;
    __shared__ double red[BS / kWave];
    const int t = threadIdx.x;
    const int64_t n = c.n;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * PER;
    for (int64_t base = (int64_t)blockIdx.x * PER; base < n; base += stride) {
        for (int64_t i = base + t; i < n && i < base + PER; i += BS) {
            const double rn = fma_t(-1.0, c.q[i], c.b[i]);
            c.r[i] = rn;
            c.p[i] = rn;
            acc = fma_t(rn, rn, acc);
        }
    }
    const double s = block_sum<BS>(acc, red);
    if (t == 0) c.part2[blockIdx.x] = s;
}

// One workgroup: rr = sum of part2 (same order as k_cg_direction) into
// sc[slot] and hist.
template <int BS>
__global__ __launch_bounds__(BS) void k_cg_record(CgLaunch c)
{
    __shared__ double red[BS / kWave];
    const double rr = sum_partials<BS>(c.part2, c.grid, red);
    if (threadIdx.x == 0) {
        c.sc[c.slot] = rr;
        *c.hist = rr;
    }
}

// hist[0, count) = 0 (the solve of an empty system).
__global__ __launch_bounds__(256) void k_cg_zero(double *hist, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) hist[i] = 0.0;
}

namespace {

template <int BS, int E, int CB>
hipError_t L_spmv_dot(const CgLaunch &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_cg_spmv_dot<BS, E, CB>), dim3((unsigned)c.spmv_grid), dim3(BS), 0, s, c);
    return hipGetLastError();
}

template <int BS, int ROWS>
hipError_t L_stencil_dot(const CgLaunch &c, hipStream_t s)
{
    const dim3 g((unsigned)c.spmv_grid);
    if (c.st.dim == 3)
        hipLaunchKernelGGL((k_cg_stencil_dot<BS, 3, ROWS>), g, dim3(BS), 0, s, c);
    else if (c.st.dim == 2)
        hipLaunchKernelGGL((k_cg_stencil_dot<BS, 2, ROWS>), g, dim3(BS), 0, s, c);
    else
        hipLaunchKernelGGL((k_cg_stencil_dot<BS, 1, ROWS>), g, dim3(BS), 0, s, c);
    return hipGetLastError();
}

template <int BS, int ROWS>
hipError_t L_stencil_lds(const CgLaunch &c, hipStream_t s)
{
    const dim3 g((unsigned)c.spmv_grid);
    const size_t sh = (size_t)stencil_lds_bytes(BS, ROWS, c.st.dim, c.st.N3, 8);
    if (c.st.dim == 3)
        hipLaunchKernelGGL((k_cg_stencil_lds<BS, 3, ROWS>), g, dim3(BS), sh, s, c);
    else if (c.st.dim == 2)
        hipLaunchKernelGGL((k_cg_stencil_lds<BS, 2, ROWS>), g, dim3(BS), sh, s, c);
    else
        hipLaunchKernelGGL((k_cg_stencil_lds<BS, 1, ROWS>), g, dim3(BS), sh, s, c);
    return hipGetLastError();
}

#define TILES(BS, E) {4, BS, E, 0, L_spmv_dot<BS, E, 4>}
#define TILES16(BS, E) {4, BS, E, 0, L_spmv_dot<BS, E, 2>, 2}
const CgEntry kCg[] = {
    TILES(128, 256), TILES(128, 512), TILES(128, 1024),
    TILES(256, 256), TILES(256, 512), TILES(256, 1024),
    TILES(512, 256), TILES(512, 512), TILES(512, 1024),
    // two-byte columns
    TILES16(256, 256), TILES16(256, 512), TILES16(512, 256), TILES16(512, 512), TILES16(512, 1024),
    TILES16(256, 1024),
    // matrix-free: `entries` = rows per lane; lds = p staged through LDS
    {6, 256, 1, 0, L_stencil_dot<256, 1>}, {6, 256, 2, 0, L_stencil_dot<256, 2>},
    {6, 256, 4, 0, L_stencil_dot<256, 4>}, {6, 512, 1, 0, L_stencil_dot<512, 1>},
    {6, 512, 2, 0, L_stencil_dot<512, 2>}, {6, 512, 4, 0, L_stencil_dot<512, 4>},
    {6, 256, 2, 1, L_stencil_lds<256, 2>}, {6, 256, 4, 1, L_stencil_lds<256, 4>},
    {6, 512, 2, 1, L_stencil_lds<512, 2>}, {6, 512, 4, 1, L_stencil_lds<512, 4>},
};
#undef TILES
#undef TILES16

}  // namespace

const CgEntry *cg_table(int *count)
{
    *count = (int)(sizeof(kCg) / sizeof(kCg[0]));
    return kCg;
}

hipError_t launch_cg_start(const CgLaunch &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_cg_start<kCgVecBlock, kCgVecUnroll>), dim3((unsigned)c.grid), dim3(kCgVecBlock), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_cg_residual(const CgLaunch &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_cg_residual<kCgVecBlock, kCgVecUnroll>), dim3((unsigned)c.grid), dim3(kCgVecBlock), 0, s,
                       c);
    return hipGetLastError();
}

hipError_t launch_cg_direction(const CgLaunch &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_cg_direction<kCgVecBlock, kCgVecUnroll>), dim3((unsigned)c.grid), dim3(kCgVecBlock), 0, s,
                       c);
    return hipGetLastError();
}

hipError_t launch_cg_record(const CgLaunch &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_cg_record<kCgVecBlock>), dim3(1), dim3(kCgVecBlock), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_cg_zero(double *hist, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, hist, count);
    return hipGetLastError();
}

}  // namespace spk
