// kernels.h -- host-visible registry of the compiled kernel variants.
//
// Each kernel family is a C++ template whose parameters are the tuning knobs
// (threads per block, lanes per row, unroll, vector width, LDS tile).  The
// instantiations compiled into the library are listed in tables; the
// dispatcher and the tuner pick entries from them at run time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_types.h"

namespace spk {

// ----------------------------------------------------------- vector kernels

struct VecLaunch {
    int64_t n;
    double alpha;
    const void *x;
    const void *y;
    void *w;             // WAXPY/AXPY output
    double *partial;     // DOT: one double per workgroup
    uint32_t *ticket;    // DOT: zero on entry, left zero on exit; null = partials
                         // only (finished by launch_dot_final)
    double *out;         // DOT: result
    int64_t grid;        // workgroups to launch
};

using VecFn = hipError_t (*)(const VecLaunch &, hipStream_t);

struct VecEntry {
    int block, vec, unroll;
    VecFn fn[2];         // [SPK_F32, SPK_F64]; null when vec*sizeof(T) > 16
};

const VecEntry *waxpy_table(int *count);
const VecEntry *dot_table(int *count);

// Second launch of a dot whose kernel ran without a ticket: *out = sum of
// partial[0, count) in a fixed order.
hipError_t launch_dot_final(const double *partial, int64_t count, double *out, hipStream_t s);

// Last pass of the column-blocked SpMV (FP64): y = sum of the nblk partials
// part[b*m + i] in block order; w = alpha*y + x when w is not null.
hipError_t launch_colblock_sum(int nblk, int64_t m, const double *part, double *y, double *w, const double *x,
                               double alpha, hipStream_t s);

// Largest dot grid finished by the ticket (each workgroup then publishes
// its partial with a device-scope release, which writes back the XCD's L2
// and serialises there); larger grids use launch_dot_final.
constexpr int64_t kDotTicketMaxGrid = 16;

// Elements covered by one workgroup in one pass.
inline int64_t vec_per_block(const VecEntry &e) { return (int64_t)e.block * e.vec * e.unroll; }

// Most work-items in one launch: a dispatch's size in work-items is a
// 32-bit quantity, so larger problems loop in the kernel (vector ops) or are
// split over several launches (SpMV row ranges).
constexpr int64_t kMaxLaunchItems = (int64_t)1 << 30;
// Most wavefront tiles in one batched launch (one wavefront per tile).
constexpr int64_t kMaxLaunchTiles = kMaxLaunchItems / 64;

// Workgroups of a vector-op launch over n elements: one pass (a workgroup
// per vec_per_block elements) or at most `per_cu` per compute unit, and in
// any case at most kMaxLaunchItems work-items; the kernels loop over the
// grid, so every n is covered.
inline int64_t vec_grid(const VecEntry &e, int64_t n, int per_cu, int num_cu)
{
    const int64_t per = vec_per_block(e);
    int64_t g = (n + per - 1) / per;
    if (per_cu > 0) g = g < (int64_t)per_cu * num_cu ? g : (int64_t)per_cu * num_cu;
    const int64_t cap = kMaxLaunchItems / e.block;
    if (g > cap) g = cap;
    return g > 1 ? g : 1;
}

// ------------------------------------------------------------- SpMV kernels

// `args` points at a SpmvArgs<T> of the entry's dtype.
using SpmvFn = hipError_t (*)(const void *args, dim3 grid, hipStream_t);

struct SpmvEntry {
    int format, block, group, unroll, lds;
    SpmvFn fn[2][2];     // [dtype][fused]
    int vec = 1;         // entries per value/index access (SCALAR, VECTOR): 1, 2 or 4; ADAPTIVE: 2 =
                         // two-byte columns in the row-stream blocks
};

const SpmvEntry *spmv_table(int *count);

// ------------------------------------------- x staged in LDS by window

// SPK_FMT_XWIN: the entries regrouped by column window (window w holds the
// columns [w*WC, (w+1)*WC), WC = window bytes / sizeof(T)) into (row,
// window) pairs, window-major and, inside a window, in row order; a pair's
// entries keep their order in the row.  Pair p has entries [ent[p],
// ent[p+1]) of ci (column inside the window) and val.  Wavefront tiles over
// the pairs never cross a window (start pair | mode << 30, as the row
// blocks of the LDS-staged kernel, and their first entries); chunk c is the
// tiles [chunk_t[c], chunk_t[c+1]) of window chunk_w[c], one workgroup each.
struct XwinArgs {
    const uint32_t *tiles;     // ntiles + 1
    const int32_t *tile_k;     // ntiles + 1
    const int32_t *chunk_t;    // nchunk + 1
    const int32_t *chunk_w;    // nchunk
    const int32_t *ent;        // npairs + 1
    const uint16_t *ci;        // nnz
    const void *val;           // T[nnz]
    const void *x;             // T[n]
    int64_t n;
    double *part;              // npairs FP64 partial sums
    int32_t nchunk;
};

using XwinFn = hipError_t (*)(const XwinArgs &a, hipStream_t s);

struct XwinEntry {
    int block, window_kib, entries;   // a variant's block, group and lds
    XwinFn fn[2];                     // [dtype]
};

const XwinEntry *xwin_table(int *count);

// Second pass, one workgroup per block of rb rows (block b = rows [b*rb,
// (b+1)*rb)): the block's partials are read run by run (window w's run
// starts at pair first[b*nwin + w] and at slot pre[b*(nwin+1) + w]) and
// placed in LDS in row order (slot j of the block goes to place
// rowpos[pos_ptr[b*rb] + j]), then y_i = the sum of row i's places (its
// pairs in window order); w_i = alpha*y_i + x_i when fused.
struct XsumArgs {
    int64_t m;
    int32_t rb, nwin;
    const int32_t *first;      // nblk * nwin
    const int32_t *pre;        // nblk * (nwin + 1)
    const int32_t *pos_ptr;    // m + 1
    const uint16_t *rowpos;    // npairs
    const double *part;        // npairs
    void *y, *w;
    const void *x;
    double alpha;
};

hipError_t launch_xwin_sum(int dtype, bool fused, const XsumArgs &a, hipStream_t s);

// ------------------------------------------------ structured SpMV formats

constexpr int kMaxDiag = 16;

// Diagonal storage: entry (row i, column i + off[d]) at val[d*m + i], present
// iff bit d of mask[i] is set.  Offsets ascend, so a row's products are
// added in ascending column order.
struct DiaArgs {
    int32_t m, ncols, ndiag;
    int32_t off[kMaxDiag];
    const void *val;           // T[ndiag*m]
    const uint16_t *mask;      // m
    const void *x;
    void *y, *w;               // w: fused step only
    double alpha;
};

// Constant-coefficient grid stencil on N1 x N2 x N3 (row r = (i*N2 + j)*N3
// + k; N1 = N2 = 1 in 1-D, N1 = 1 in 2-D).  coef[] holds the values of the
// offsets -N2*N3, -N3, -1, 0, +1, +N3, +N2*N3 in that (ascending) order;
// a neighbour outside the grid is absent.
struct StencilArgs {
    int32_t n, N1, N2, N3, dim;
    double coef[7];
    const void *x;
    void *y, *w;
    double alpha;
};

using StructFn = hipError_t (*)(const void *args, hipStream_t);

struct StructEntry {
    int format, block, rows;   // rows per lane (a variant's `unroll`)
    int lds;                   // stencil: 1 = x staged through LDS (a variant's `lds`)
    StructFn fn[2][2];         // [dtype][fused]
};

// LDS-staged stencil kernels keep a workgroup's rows plus one grid line of
// halo on each side (block*rows + 2*N3 values, 2 in 1-D) in LDS; they apply
// while that fits this budget.
constexpr int64_t kStencilLdsMaxBytes = 64 * 1024;
inline int64_t stencil_lds_bytes(int block, int rows, int dim, int N3, int elem)
{
    const int64_t halo = dim >= 2 ? N3 : 1;
    return ((int64_t)block * rows + 2 * halo) * elem;
}

const StructEntry *struct_table(int *count);

// val_dia[d*m + i] and mask[i] from CSR (val_dia zeroed by the caller).
hipError_t launch_csr_to_dia(int dtype, int32_t m, const int32_t *rp, const int32_t *ci, const void *val,
                             int32_t ndiag, const int32_t *off_host, void *val_dia, uint16_t *mask, hipStream_t s);

// --------------------------------------------------------- batched kernels

using BatchFn = hipError_t (*)(const void *args, dim3 grid, hipStream_t);

// Launch kinds of the batched kernel.  Tiles are wavefront-sized: a
// workgroup of BS threads runs BS/64 consecutive tiles, one per wavefront.
constexpr int kBatchGrid = 0;        // one workgroup per group of BS/64 tiles
constexpr int kBatchPersistent = 1;  // persistent grid pulling tile groups from per-XCD queues

struct BatchEntry {
    int block, tile;     // threads per workgroup, LDS products per workgroup
    int xw;              // LDS room for x per wavefront (entries) for mode-1 tiles, 0 = none
    BatchFn fn[2][2];    // [dtype][launch kind]
    int (*occupancy[2])();  // [dtype] resident workgroups per CU (persistent kernel)
};

const BatchEntry *batch_table(int *count);

// Row-stream capacity (entries) of one wavefront's tile.
inline int batch_wave_entries(const BatchEntry &e) { return e.tile / (e.block / 64); }

// The x windows of mode-1 and mode-3 tiles: for each such tile with
// entries, the smallest and largest column of its entries; the window is
// recorded (xlo, xn) when it spans at most `cap` columns, else xn = 0.
// Mode-3 tiles (compact columns): one whose window fits (cap <= 256)
// writes its entries' offsets in the window, one byte each, to c8 at the
// place its column array ci0 + d has (c8 + d), and points its ci there;
// one whose columns span at most 65,536 writes two-byte offsets from its
// first column (xlo) to c16 the same way and becomes a mode-5 tile, or,
// with c16 NULL, adds 1 to *need16 (when not NULL) and becomes a mode-1
// tile; any other becomes a mode-1 tile.  One wavefront per tile.
hipError_t launch_tile_windows(BatchTile *tiles, int64_t ntiles, int cap, hipStream_t s,
                               const int32_t *ci0 = nullptr, uint8_t *c8 = nullptr, uint16_t *c16 = nullptr,
                               int *need16 = nullptr);

// The same for the row-stream blocks of the single-matrix row-block kernel:
// bx[2b], bx[2b+1] = first column and length of block b's window (length 0
// for other blocks and for windows wider than `cap`).
hipError_t launch_block_windows(const uint32_t *blocks, const int32_t *block_k, const int32_t *ci, int32_t nblk,
                                int cap, int32_t *bx, hipStream_t s);

// Two-byte columns of the row-block kernel: for each row-stream block with
// entries whose columns span at most 65,536, base[b] = its smallest column
// and c16[k] = ci[k] - base[b] over its entries; base[b] = -1 for every
// other block (c16 is then not written for its entries).
hipError_t launch_block_c16(const uint32_t *blocks, const int32_t *block_k, const int32_t *ci, int32_t nblk,
                            uint16_t *c16, int32_t *base, hipStream_t s);

// ------------------------------------------------------ conjugate gradients

// Device scalars of one solve: r.r of the current iteration alternates
// between sc[0] and sc[1] (the slot of iteration k is k & 1), so a kernel
// can read one while its first workgroup writes the other; sc[kCgAlpha]
// carries alpha from the residual kernel to the direction kernel.
constexpr int kCgAlpha = 2, kCgScalars = 3;
constexpr int kCgVecBlock = 256, kCgVecUnroll = 4;
constexpr int64_t kCgVecPer = (int64_t)kCgVecBlock * 2 * kCgVecUnroll;   // elements per workgroup pass

struct CgLaunch {
    int64_t n;                 // rows (= columns)
    const int32_t *rp, *ci;    // CSR of the matrix
    const double *val;
    const uint32_t *blocks;    // wavefront tiles: nblk + 1 packed starts
    const int32_t *block_k;    // first entry of each tile
    int32_t nblk;
    int32_t spmv_grid;         // workgroups of the SpMV kernel = tile groups (slots of part1)
    const double *spmv_x;      // operand of the product (p, or x at the start)
    const double *b;
    double *x, *r, *p, *q;     // x, r, p, q 16-byte aligned
    double *part1;             // p.q partials, one per SpMV workgroup (null: no dot)
    double *part2;             // r.r partials, one per vector workgroup
    double *sc;                // kCgScalars doubles
    double *hist;              // where this launch records r.r
    const uint16_t *c16;       // two-byte columns of the tiles (entries with vec 2), else null
    const int32_t *block_c16;  // base column of each tile's two-byte columns, -1 = none
    int32_t slot;              // iteration parity
    int64_t grid;              // workgroups of the vector kernels (slots of part2)
    StencilArgs st;            // stencil form of the matrix (SpMV+dot of a STENCIL entry)
};

using CgFn = hipError_t (*)(const CgLaunch &, hipStream_t);

// An SpMV+dot kernel of the solve: SPK_FMT_ADAPTIVE (CSR wavefront tiles of
// `entries` entries, one workgroup per tile group) or SPK_FMT_STENCIL
// (matrix-free, grid-stride rows, `entries` rows per lane).
struct CgEntry {
    int format, block, entries;
    int lds;                   // matrix-free: 1 = p staged through LDS
    CgFn spmv_dot;
    int vec = 0;               // tiles: 2 = two-byte columns in the row-stream tiles
};

const CgEntry *cg_table(int *count);
hipError_t launch_cg_start(const CgLaunch &c, hipStream_t s);
hipError_t launch_cg_residual(const CgLaunch &c, hipStream_t s);
hipError_t launch_cg_direction(const CgLaunch &c, hipStream_t s);
hipError_t launch_cg_record(const CgLaunch &c, hipStream_t s);
hipError_t launch_cg_zero(double *hist, int64_t count, hipStream_t s);

// ------------------------------------------------------------- utilities

// Counts outputs that fail the acceptance test against a reference held in
// double: mode 0 = per-element |out - ref| <= tau*scale (scale null -> 0),
// mode 1 = ulp distance <= 1 after rounding ref to T.  NaN/Inf must match.
hipError_t launch_check(int dtype, int mode, int64_t n, const void *out, const double *ref,
                        const double *scale, double tau, unsigned long long *bad, hipStream_t s);

// out[i] = (double)in[i]
hipError_t launch_widen(int dtype, int64_t n, const void *in, double *out, hipStream_t s);

// scale_i = sum_k |a_ik * x_k| over rows [0, m)
hipError_t launch_row_absum(int dtype, int32_t m, const int32_t *rp, const int32_t *ci,
                            const void *val, const void *x, double *scale, hipStream_t s);

// scale[vec_off + r] = sum_k |a_rk * x_k| for every row of every tile
hipError_t launch_tiles_absum(int dtype, const BatchTile *tiles, int64_t ntiles, const void *x, double *scale,
                              hipStream_t s);

// scale_i = |x_i * y_i| summed into one double (dot tolerance scale)
hipError_t launch_dot_absum(int dtype, int64_t n, const void *x, const void *y, double *out,
                            hipStream_t s);

// Sets n 32-bit words to zero (a kernel: capture-safe, unlike a memset node).
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);

// Fills n bytes (n a multiple of 16) with a pattern: evicts caches.
hipError_t launch_fill(void *p, int64_t n, uint32_t pattern, hipStream_t s);

// Reads n bytes (a multiple of 16) so the caches hold clean lines of p;
// `sink` (16 bytes) is written only in a case that never occurs.
hipError_t launch_evict(const void *p, int64_t n, void *sink, hipStream_t s);

// STREAM copy (b = a) and triad (c = a + s*b) on doubles.
hipError_t launch_copy(int64_t n, const double *a, double *b, hipStream_t s);
hipError_t launch_triad(int64_t n, const double *a, const double *b, double s_, double *c,
                        hipStream_t s);

// Counts malformed CSR entries: columns outside [0, ncols).
hipError_t launch_csr_colcheck(int64_t nnz, const int32_t *ci, int64_t ncols,
                               unsigned long long *bad, hipStream_t s);

// Scatters CSR rows into sliced-ELL storage (C rows per slice).
hipError_t launch_csr_to_sell(int dtype, int32_t m, int32_t C, const int32_t *rp, const int32_t *ci,
                              const void *val, const int64_t *sell_ptr, int32_t *sell_len,
                              int32_t *sell_ci, void *sell_val, hipStream_t s);

}  // namespace spk
