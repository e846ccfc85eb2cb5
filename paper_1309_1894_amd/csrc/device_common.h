// device_common.h -- wavefront primitives and argument blocks shared by the
// gfx950 kernels of libspk.
//
// Every reduction here has a fixed combination order, so a given kernel
// variant produces bit-identical results on every run, alone or batched.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_types.h"
#include "row_tiles.h"

namespace spk {

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------- FP helpers

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Vector of N elements loaded/stored as one 4/8/16-byte access.
template <typename T, int N>
struct alignas(sizeof(T) * N) vec_t {
    T v[N];
};

// ------------------------------------------------------- lane data movement
//
// DPP moves 32-bit lanes; a double travels as two halves.  update_dpp with
// old = 0 and bound_ctrl set yields 0 for a source lane outside the pattern
// (none of the patterns below has one).

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// ds_swizzle in bit mode (offset bit 15 clear): within each group of 32
// lanes, lane i reads lane ((i & and) | or) ^ xor.
template <int PATTERN>
__device__ __forceinline__ double swizzle_f64(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)(u & 0xffffffffull), PATTERN);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(u >> 32), PATTERN);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// DPP control codes (GFX9 encoding).
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;   // lane 15-i within each row of 16
constexpr int kDppHalfMirror = 0x141;  // lane 7-i within each half-row of 8
constexpr int kSwzXor16 = 0x401F;      // and 0x1F, or 0, xor 0x10

// Sum over aligned groups of G lanes (G a power of two, 1..64).  Every lane
// of a group receives the same bits: each step adds a lane's value to its
// partner's, and IEEE addition is commutative, so partners agree.
// All lanes of the wavefront must be active.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "G");
    if constexpr (G >= 2) v += dpp_f64<kDppXor1>(v);
    if constexpr (G >= 4) v += dpp_f64<kDppXor2>(v);
    // After the quad steps every lane of a quad holds the quad's sum; the
    // half-row mirror pairs each lane with a lane of the other quad.
    if constexpr (G >= 8) v += dpp_f64<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_f64<kDppRowMirror>(v);
    if constexpr (G >= 32) v += swizzle_f64<kSwzXor16>(v);
    if constexpr (G >= 64) v = readlane_f64(v, 0) + readlane_f64(v, 32);
    return v;
}

// Block-wide sum; `red` holds BS/64 doubles of LDS.  Returns the total to
// every thread.  Waves are combined in index order.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    constexpr int NW = BS / kWave;
    v = group_sum<kWave>(v);
    if constexpr (NW == 1) {
        return v;
    } else {
        const int wid = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) red[wid] = v;
        __syncthreads();
        double t = red[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t += red[i];
        __syncthreads();
        return t;
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b % 8), each XCD with its own L2.
constexpr int kXcds = 8;

// XCD k's contiguous eighth of n items starts at xcd_first(k, n).
__device__ __forceinline__ int xcd_first(int xcd, int n)
{
    const int per = n / kXcds, rem = n % kXcds;
    return xcd * per + min(xcd, rem);
}

// Chunked dealing: the n items are cut into runs of C, and the runs go to
// the XCDs in turn (run j to XCD j % 8), in order.  Every XCD meets
// neighbouring items together (inside a run, so rows that share x entries
// share an L2), and all eight stream the same region of the arrays at any
// time, with equal shares of it.  Contiguous eighths per XCD were slower:
// 5% on the batched tile kernel, whose tiles differ in bytes so that some
// eighths hold more than others, and 1-3% on the single-matrix row-block
// and CG kernels.  Items past the last whole round of 8*C keep b (plain
// round-robin).  A bijection on [0, n) for any C >= 1.
__device__ __forceinline__ int xcd_chunk(int b, int n, int C)
{
    const int full = n / (kXcds * C) * (kXcds * C);
    if (b >= full) return b;
    const int i = b / kXcds;
    return (b % kXcds + kXcds * (i / C)) * C + i % C;
}

constexpr int kXcdRunGroups = 16;   // workgroups per run for the row-block kernels

__device__ __forceinline__ int xcd_remap(int b, int n) { return xcd_chunk(b, n, kXcdRunGroups); }

// ------------------------------------------------------------ SpMV operands

// One launch of a SpMV kernel over the row range [row0, row0 + m) (or, for
// the row-block kernel, over row blocks [blk0, blk0 + nblk)).
template <typename T>
struct SpmvArgs {
    int32_t row0, m;
    const int32_t *rp;     // CSR row_ptr (global row indexing)
    const int32_t *ci;     // CSR col_idx
    const T *val;          // CSR values
    const T *x;
    T *y;
    T *w;                  // fused step output (w = alpha*y + x), else null
    T alpha;
    // sliced ELL
    const int64_t *sell_ptr;   // first entry of each slice
    const int32_t *sell_len;   // stored entries per row
    const int32_t *sell_ci;
    const T *sell_val;
    // row blocks (LDS-staged kernel): start row | mode << 30 and first entry,
    // nblk + 1 entries each
    const uint32_t *blocks;
    const int32_t *block_k;
    const int32_t *block_x;   // row-stream blocks' x windows (first column, length; length 0 = none), or null
    const uint16_t *c16;      // two-byte columns: each row-stream entry's column minus its block's base
    const int32_t *block_c16; // base (first column) of each block with two-byte columns, -1 = none
    int32_t blk0, nblk;
};

// Row blocks of the LDS-staged kernel are wavefront tiles:

// ------------------------------------------------------------ batched tiles

template <typename T>
struct BatchArgs {
    const BatchTile *tiles;
    int32_t ntiles;
    const T *x;
    T *y;
    T *w;              // may be null (SpMV only)
    T alpha;
    uint32_t *next;    // tile queue head (persistent launch), zero between launches
    uint32_t *done;    // finished workgroups (persistent launch), zero between launches
    const BatchReq *reqs;            // serving (grid launch): tiles named per request, or null
    const uint16_t *req_of_tile;     // request of each launch tile (with reqs)
};

}  // namespace spk
