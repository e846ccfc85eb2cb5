// kernels_batch.hip -- one launch over many independent CSR instances.
//
// The host planner cuts every instance into tiles (row ranges) and gives
// each tile the kernel chosen for the instance's shape class: an LDS-staged
// row stream (mode 0) or G lanes per row (mode G).  The kernel either runs
// one workgroup per group of tiles (one tile per wavefront), or is
// persistent: a grid sized to fill the GPU pulls tiles from queue heads in
// device memory until the queues are empty.
// The queue head and a completion counter are left at zero by the last
// workgroup to finish, so the launch can be captured in a hipGraph and
// replayed without a reset node.
//
// Each row is always reduced by the same code in the same order, so a
// row's result depends only on (matrix, tile mode): an instance gives the
// same bits alone, in a batch, or in any other mix.
#include "device_common.h"
#include "device_rows.h"
#include "kernels.h"

namespace spk {

// Tiles per run when tile groups are dealt to the XCDs (measured on the
// 4096-instance banded batch: runs of 32 to 128 tiles stream 5% faster than
// contiguous eighths, and 2-3% faster than dealing single groups).
constexpr int kXcdRunTiles = 64;

// Tiles are wavefront-sized: every wavefront of a workgroup runs its own
// tile, with its own slice of the workgroup's LDS (TILE/(BS/64) products and
// 129 row offsets), and no workgroup barrier.
template <typename T, int BS, int TILE>
struct WaveTiles {
    static constexpr int NW = BS / kWave;        // wavefronts per workgroup
    static constexpr int ENTRIES = TILE / NW;    // row-stream capacity of one wavefront
    static constexpr int ITEMS = ENTRIES / kWave;
    static_assert(ITEMS * kWave * NW == TILE, "tile must split evenly over the wavefronts");
};

template <typename T, int BS, int TILE, int XW>
__device__ __forceinline__ void run_wave_tile(const BatchArgs<T> &a, const BatchTile &td, double *sp, int *srp, T *xs)
{
    const int32_t *rp = td.rp;
    const int32_t *ci = td.ci;
    const T *val = (const T *)td.val;
    const T *x = a.x + td.vec_off;
    T *y = a.y + td.vec_off;
    T *w = a.w ? a.w + td.vec_off : nullptr;
    switch (td.mode) {
    case 0:  // entries and rows fit the wavefront's LDS slice (guaranteed by the planner)
        wave_stream<T, WaveTiles<T, BS, TILE>::ITEMS>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1, td.k0, td.k1,
                                                      sp, srp);
        break;
    case 1:  // the same, x from the tile's window in LDS when it fits the kernel's room
        wave_stream<T, WaveTiles<T, BS, TILE>::ITEMS, false, XW>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1,
                                                                 td.k0, td.k1, sp, srp, td.xlo,
                                                                 XW > 0 && td.xn <= XW ? td.xn : 0, xs);
        break;
    case 3:  // mode 1 with compact columns: ci holds each entry's byte offset in the window (which fits)
        if constexpr (XW > 0 && XW <= 256)
            wave_stream<T, WaveTiles<T, BS, TILE>::ITEMS, false, XW, 1>(rp, ci, val, x, y, w, a.alpha, td.r0,
                                                                           td.r1, td.k0, td.k1, sp, srp, td.xlo,
                                                                           td.xn, xs);
        break;
    case 5:  // compact columns of a wider tile: two-byte offsets from xlo, x gathered from memory
        wave_stream<T, WaveTiles<T, BS, TILE>::ITEMS, false, XW, 2>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1,
                                                                       td.k0, td.k1, sp, srp, td.xlo, 0, xs);
        break;
    case 2: wave_group_rows<T, 2>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 4: wave_group_rows<T, 4>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 8: wave_group_rows<T, 8>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 16: wave_group_rows<T, 16>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 32: wave_group_rows<T, 32>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    default: wave_group_rows<T, 64>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    }
}

template <typename T, int BS, int TILE, int XW>
__global__ __launch_bounds__(BS) void k_batch_grid(BatchArgs<T> a)
{
    using WT = WaveTiles<T, BS, TILE>;
    __shared__ double sp[TILE];
    __shared__ int srp[WT::NW * (kWaveTileRows + 1)];
    __shared__ T xs[WT::NW * (XW > 0 ? XW : 1)];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int ngroups = (a.ntiles + WT::NW - 1) / WT::NW;
    const int b = (int)blockIdx.x;
    // runs of kXcdRunTiles tiles dealt to the XCDs in turn
    const int tile = xcd_chunk(b, ngroups, kXcdRunTiles / WT::NW) * WT::NW + wv;
    if (tile >= a.ntiles) return;
    // the tile record stays wavefront-uniform: the 16-bit map entry arrives
    // through a vector load and is made uniform again
    const BatchTile *tp = a.tiles + tile;
    int64_t voff = -1;
    if (a.req_of_tile) {
        const int r = __builtin_amdgcn_readfirstlane((int)a.req_of_tile[tile]);
        const BatchReq *q = a.reqs + r;
        tp = q->tiles + (tile - q->first);
        voff = q->vec_off;
    }
    // the address made uniform and read through the constant address space:
    // scalar loads, as for a tile array passed in the arguments
    const uint64_t ta = (uint64_t)tp;
    const uint64_t tu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(ta >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)ta);
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const __attribute__((address_space(4))) u32x4 *src = (const __attribute__((address_space(4))) u32x4 *)tu;
    u32x4 parts[sizeof(BatchTile) / sizeof(u32x4)];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BatchTile) / sizeof(u32x4)); ++i) parts[i] = src[i];
    BatchTile td;
    __builtin_memcpy(&td, parts, sizeof td);
    if (voff >= 0) td.vec_off = voff;
    run_wave_tile<T, BS, TILE, XW>(a, td, sp + wv * WT::ENTRIES, srp + wv * (kWaveTileRows + 1),
                                   xs + wv * (XW > 0 ? XW : 1));
}

// Persistent form: a grid sized to fill the GPU whose wavefronts pull tiles
// themselves: a wavefront on XCD k claims chunks of kChunk tiles from XCD
// k's own eighth of the tile list (one queue head per XCD, each in its own
// 256-byte line) and streams them; no workgroup barrier anywhere.
constexpr int kChunk = 4;
constexpr int kCtrStride = 64;   // uint32 per counter line

template <typename T, int BS, int TILE, int XW>
__global__ __launch_bounds__(BS) void k_batch_persistent(BatchArgs<T> a)
{
    using WT = WaveTiles<T, BS, TILE>;
    __shared__ double sp[TILE];
    __shared__ int srp[WT::NW * (kWaveTileRows + 1)];
    __shared__ T xs[WT::NW * (XW > 0 ? XW : 1)];
    const int l = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int xcd = (int)blockIdx.x % kXcds;
    const int lo = xcd_first(xcd, a.ntiles);
    const int hi = xcd_first(xcd + 1, a.ntiles);
    uint32_t *head = a.next + xcd * kCtrStride;
    double *my_sp = sp + wv * WT::ENTRIES;
    int *my_srp = srp + wv * (kWaveTileRows + 1);
    T *my_xs = xs + wv * (XW > 0 ? XW : 1);
    // the next claim is issued before the current chunk is streamed, so the
    // atomic's round trip overlaps the chunk's loads
    int claim = 0;
    if (l == 0) claim = (int)atomicAdd(head, (uint32_t)kChunk);
    for (;;) {
        const int c0 = lo + __builtin_amdgcn_readlane(claim, 0);
        if (c0 >= hi) break;
        if (l == 0) claim = (int)atomicAdd(head, (uint32_t)kChunk);
        const int c1 = min(c0 + kChunk, hi);
        for (int tile = c0; tile < c1; ++tile) run_wave_tile<T, BS, TILE, XW>(a, a.tiles[tile], my_sp, my_srp, my_xs);
    }
    // Every wavefront has drawn past the end of its queue before it counts
    // itself done, so the last one may reset all counters.  Only atomics
    // are involved, and each one this wavefront issued has returned its
    // value (it decided the exit) before the done count is incremented, so
    // no fence is needed; a device-scope release here would write back the
    // XCD's L2 once per wavefront, serialised per XCD.
    if (l == 0) {
        const uint32_t d = atomicAdd(a.done, 1u);
        if (d == gridDim.x * (uint32_t)WT::NW - 1u) {
            for (int k = 0; k < kXcds; ++k) atomicExch(a.next + k * kCtrStride, 0u);
            atomicExch(a.done, 0u);
        }
    }
}

// The x windows of mode-1 and mode-3 tiles (see launch_tile_windows), one
// wavefront per tile.  A mode-3 tile whose window fits writes its entries'
// offsets in the window to c8 (at the entries' own positions: instance
// arrays at ci + d map to c8 + d) and takes c8 as its column array; one
// whose columns span at most 65,536 does the same with two-byte offsets
// from its first column in c16 and becomes a mode-5 tile (x gathered from
// memory), or, while c16 is NULL, counts itself in *need16 and becomes a
// mode-1 tile; any other becomes a mode-1 tile.
__global__ __launch_bounds__(256) void k_tile_windows(BatchTile *tiles, int64_t ntiles, int cap, const int32_t *ci0,
                                                      uint8_t *c8, uint16_t *c16, int *need16)
{
    const int64_t t = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (t >= ntiles) return;
    const int l = threadIdx.x & (kWave - 1);
    BatchTile &td = tiles[t];
    const int mode = td.mode;
    if (mode != 1 && mode != 3) return;
    const int32_t *ci = td.ci;
    const int k0 = td.k0, k1 = td.k1;
    int lo = INT32_MAX, hi = -1;
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
    const bool fits = hi >= lo && (int64_t)hi - lo + 1 <= cap;
    const bool span16 = hi >= lo && (int64_t)hi - lo < 65536;
    const bool one = mode == 3 && fits && cap <= 256 && c8 != nullptr;
    const bool two = mode == 3 && !one && span16 && c16 != nullptr;
    uint8_t *cb = one ? c8 + (ci - ci0) : nullptr;
    uint16_t *cw = two ? c16 + (ci - ci0) : nullptr;
    if (one)
        for (int k = k0 + l; k < k1; k += kWave) cb[k] = (uint8_t)(ci[k] - lo);
    if (two)
        for (int k = k0 + l; k < k1; k += kWave) cw[k] = (uint16_t)(ci[k] - lo);
    if (l == 0) {
        td.xlo = fits || two ? lo : 0;
        td.xn = fits && !two ? hi - lo + 1 : 0;
        if (mode == 3) {
            td.mode = one ? 3 : two ? 5 : 1;
            if (one) td.ci = reinterpret_cast<const int32_t *>(cb);
            if (two) td.ci = reinterpret_cast<const int32_t *>(cw);
            if (!one && !two && span16 && c16 == nullptr && need16 != nullptr) atomicAdd(need16, 1);
        }
    }
}

namespace {

template <typename T, int BS, int TILE, int XW>
int occ_batch()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_batch_persistent<T, BS, TILE, XW>),
                                                     BS, 0) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

template <typename T, int BS, int TILE, int XW, int KIND>
hipError_t L_batch(const void *p, dim3 g, hipStream_t s)
{
    if constexpr (KIND == 1)
        hipLaunchKernelGGL((k_batch_persistent<T, BS, TILE, XW>), g, dim3(BS), 0, s, *(const BatchArgs<T> *)p);
    else
        hipLaunchKernelGGL((k_batch_grid<T, BS, TILE, XW>), g, dim3(BS), 0, s, *(const BatchArgs<T> *)p);
    return hipGetLastError();
}

#define BENTRY(BS, TILE, XW)                                                                 \
    {BS, TILE, XW,                                                                           \
     {{L_batch<float, BS, TILE, XW, 0>, L_batch<float, BS, TILE, XW, 1>},                    \
      {L_batch<double, BS, TILE, XW, 0>, L_batch<double, BS, TILE, XW, 1>}},                 \
     {occ_batch<float, BS, TILE, XW>, occ_batch<double, BS, TILE, XW>}}

// (threads per workgroup, LDS products per workgroup, LDS room for x per
// wavefront): a wavefront's row stream holds TILE/(BS/64) entries: 256
// to 2048; the kernels with room for x run mode-1 tiles from LDS
const BatchEntry kBatch[] = {
    BENTRY(256, 2048, 0), BENTRY(256, 1024, 0), BENTRY(256, 4096, 0),
    BENTRY(128, 1024, 0), BENTRY(128, 2048, 0),
    BENTRY(512, 2048, 0), BENTRY(512, 4096, 0),
    BENTRY(256, 2048, 256), BENTRY(256, 4096, 256), BENTRY(128, 2048, 256),
    BENTRY(128, 1024, 256), BENTRY(64, 1024, 256), BENTRY(64, 512, 256), BENTRY(64, 2048, 256),
};

}  // namespace

const BatchEntry *batch_table(int *count)
{
    *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
    return kBatch;
}

hipError_t launch_tile_windows(BatchTile *tiles, int64_t ntiles, int cap, hipStream_t s, const int32_t *ci0,
                               uint8_t *c8, uint16_t *c16, int *need16)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_windows, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, tiles, ntiles, cap, ci0,
                       c8, c16, need16);
    return hipGetLastError();
}

}  // namespace spk
