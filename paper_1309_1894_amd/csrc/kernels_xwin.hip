// kernels_xwin.hip -- CSR SpMV with x staged in LDS by column window
// (SPK_FMT_XWIN).
//
// A random-column matrix gathers x from all over the vector; once x is
// larger than an XCD's L2, most gathers miss it and each miss moves a whole
// 128-byte line for 8 useful bytes.  Here the columns are cut into windows
// of at most 128 KiB of x (64 KiB for the smaller variants), small enough to
// live in a compute unit's LDS.  At conversion the entries are regrouped
// window by window: a (row, window) pair holds the row's entries whose
// columns fall in the window, in their original order, with 16-bit column
// indices inside the window.  The first pass runs one workgroup per chunk of
// one window's pairs: it copies that window of x into LDS once, then its
// wavefronts stream the pairs' values and indices with coalesced loads,
// take x from LDS and write one FP64 partial per pair.  A second pass adds
// each row's partials in window order (and forms w = alpha*y + x when
// fused).  Every byte of the first pass is a coalesced stream; the gathers
// never leave the compute unit.
#include "device_common.h"
#include "device_rows.h"
#include "kernels.h"
#include "xwin_layout.h"

namespace spk {

namespace {

// One wavefront tile: pairs [p0, p1) with entries [k0, k1); a row-stream
// tile (k1 - k0 <= 64*ITEMS, p1 - p0 <= 128) carries its lanes' indices,
// values and pair starts, loaded ahead of its processing.
template <typename T, int ITEMS>
struct WinTile {
    int p0, p1, k0, k1;
    bool stream;
    uint16_t c[ITEMS];
    T v[ITEMS];
    int rpv[3];
};

// Takes a tile's record (start pair | mode << 30, first entry, and the
// next tile's) and issues the loads of its first 64*ITEMS entries and of
// its pair starts, whatever the tile's mode (a tile holds at least one pair
// and every pair at least one entry, so these stay inside the tile; lanes
// past its end load its last entry again and drop it).  Loading
// unconditionally keeps the pipeline's load counts fixed.
template <typename T, int ITEMS>
__device__ __forceinline__ void window_load(const XwinArgs &a, uint32_t e0, uint32_t e1, int k0, int k1,
                                            WinTile<T, ITEMS> &tl)
{
    tl.p0 = (int)(e0 & kBlkRowMask);
    tl.p1 = (int)(e1 & kBlkRowMask);
    tl.k0 = k0;
    tl.k1 = k1;
    tl.stream = (e0 >> 30) == kBlkStream;
    const gptr<int32_t> ent = as_global(a.ent);
    const gptr<uint16_t> ci = as_global(a.ci);
    const gptr<T> val = as_global((const T *)a.val);
    const int l = threadIdx.x & (kWave - 1);
    const int np = tl.p1 - tl.p0, klast = tl.k1 - tl.k0 - 1;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) tl.c[j] = __builtin_nontemporal_load(ci + tl.k0 + min(l + j * kWave, klast));
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) tl.v[j] = __builtin_nontemporal_load(val + tl.k0 + min(l + j * kWave, klast));
    // raw pair starts: k0 is taken off where they are used, so that no
    // arithmetic here has to wait for the loads
#pragma unroll
    for (int q = 0; q < 3; ++q) tl.rpv[q] = ent[tl.p0 + min(l + q * kWave, np)];
}

// Row-stream tile: products (x from the window in LDS) to the wavefront's
// LDS slice sp, then one lane per pair adds that pair's products (four
// interleaved partial sums) and writes its partial.
template <typename T, int ITEMS>
__device__ __forceinline__ void window_stream(const XwinArgs &a, const T *win, const WinTile<T, ITEMS> &tl,
                                              double *sp, int *srp)
{
    const gptr_mut<double> part = as_global_mut(a.part);
    const int l = threadIdx.x & (kWave - 1);
    const int np = tl.p1 - tl.p0;
    // stores without branches where the slice has room: products of lanes
    // past the tile's end (loaded from the clamped last entry) and pair
    // starts past np land in slots no pair sum reads
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) sp[l + j * kWave] = (double)tl.v[j] * (double)win[tl.c[j]];
#pragma unroll
    for (int q = 0; q < 2; ++q) srp[l + q * kWave] = tl.rpv[q] - tl.k0;
    if (l + 2 * kWave <= np) srp[l + 2 * kWave] = tl.rpv[2] - tl.k0;
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = l + q * kWave;
        if (i < np) {
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
            __builtin_nontemporal_store((a0 + a1) + (a2 + a3), part + tl.p0 + i);
        }
    }
    wave_lds_sync();   // the slice is free again for the next tile
}

// Pairs [p0, p1) one after another, all 64 lanes on each: UNR loads per lane
// in flight, UNR partial sums combined in a fixed order, then the wavefront
// sum.
template <typename T, int UNR>
__device__ __forceinline__ void window_pairs(const XwinArgs &a, const T *win, int p0, int p1)
{
    const gptr<int32_t> ent = as_global(a.ent);
    const gptr<uint16_t> ci = as_global(a.ci);
    const gptr<T> val = as_global((const T *)a.val);
    const int l = threadIdx.x & (kWave - 1);
    for (int p = p0; p < p1; ++p) {
        const int s = ent[p], e = ent[p + 1];
        double acc[UNR];
#pragma unroll
        for (int j = 0; j < UNR; ++j) acc[j] = 0.0;
        for (int base = s; base < e; base += kWave * UNR) {
            uint16_t c[UNR];
            T v[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int k = min(base + l + j * kWave, e - 1);
                c[j] = __builtin_nontemporal_load(ci + k);
                v[j] = __builtin_nontemporal_load(val + k);
            }
#pragma unroll
            for (int j = 0; j < UNR; ++j)
                if (base + l + j * kWave < e) acc[j] = fma_t((double)v[j], (double)win[c[j]], acc[j]);
        }
#pragma unroll
        for (int d = 1; d < UNR; d *= 2)
#pragma unroll
            for (int j = 0; j + d < UNR; j += 2 * d) acc[j] += acc[j + d];
        const double sum = group_sum<kWave>(acc[0]);
        if (l == 0) a.part[p] = sum;
    }
}

}  // namespace

// First pass: workgroup c runs chunk c, tiles [chunk_t[c], chunk_t[c+1]) of
// window chunk_w[c]; wavefront v takes tiles v, v + NW, ...  The window's
// x values (WB bytes at most) are copied to LDS once, eight loads in flight
// per lane.
constexpr int kRing = 4;   // tiles in the window pass's software pipeline

template <typename T, int BS, int WB, int E>
__global__ __launch_bounds__(BS) void k_xwin(XwinArgs a)
{
    constexpr int NW = BS / kWave;
    constexpr int WC = WB / (int)sizeof(T);
    __shared__ T win[WC];
    __shared__ double sp[NW * E];
    __shared__ int srp[NW * (kWaveTileRows + 1)];
    const int c = (int)blockIdx.x;
    const int wnd = a.chunk_w[c];
    const int64_t col0 = (int64_t)wnd * WC;
    const int ncw = (int)min<int64_t>((int64_t)WC, a.n - col0);
    const T *xs = (const T *)a.x + col0;
    constexpr int BATCH = 8;
    for (int i0 = 0; i0 < ncw; i0 += BS * BATCH) {
        T t[BATCH];
        // clamped, so the loads are issued unconditionally (a chunk's window
        // holds at least one column)
#pragma unroll
        for (int j = 0; j < BATCH; ++j) t[j] = xs[min(i0 + j * BS + (int)threadIdx.x, ncw - 1)];
#pragma unroll
        for (int j = 0; j < BATCH; ++j) {
            const int i = i0 + j * BS + (int)threadIdx.x;
            if (i < ncw) win[i] = t[j];
        }
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int t1 = a.chunk_t[c + 1];
    double *my_sp = sp + wv * E;
    int *my_srp = srp + wv * (kWaveTileRows + 1);
    // The wavefront's tiles are t0, t0 + NW, ...; their records are read 64
    // at a time with one vector load per lane (kept in registers and taken
    // out with readlane, so no scalar load stands between a tile and its
    // data), then the tiles run as a software pipeline over a ring of
    // kRing: the loads of the next kRing - 1 tiles are in flight while one
    // is summed (seven loads per tile: within the 63 a wavefront may have
    // outstanding; a ring of eight ran slower).
    using Tile = WinTile<T, E / kWave>;
    const int l = threadIdx.x & (kWave - 1);
    const int tw0 = a.chunk_t[c] + wv;
    const int ntw = tw0 < t1 ? (t1 - tw0 + NW - 1) / NW : 0;
    for (int bt = 0; bt < ntw; bt += kWave) {
        const int nb = min(kWave, ntw - bt);
        uint32_t r0 = 0, r1 = 0;
        int q0 = 0, q1 = 0;
        if (l < nb) {
            const int ti = tw0 + (bt + l) * NW;
            r0 = a.tiles[ti];
            r1 = a.tiles[ti + 1];
            q0 = a.tile_k[ti];
            q1 = a.tile_k[ti + 1];
        }
        // tile i of the batch (clamped to the last: the pipeline's loads
        // are issued unconditionally)
        auto load = [&](int i, Tile &tl) {
            i = min(i, nb - 1);
            window_load(a, (uint32_t)__builtin_amdgcn_readlane((int)r0, i), (uint32_t)__builtin_amdgcn_readlane((int)r1, i),
                        __builtin_amdgcn_readlane(q0, i), __builtin_amdgcn_readlane(q1, i), tl);
        };
        // row-stream tiles through the pipeline (their processing issues
        // no loads, so the pipeline's waits stay exact) ...
        auto run = [&](const Tile &tl) {
            if (tl.stream) window_stream(a, win, tl, my_sp, my_srp);
        };
        // ring slots are indexed by constants once the inner loop is
        // unrolled, so the ring stays in registers
        Tile ring[kRing];
#pragma unroll
        for (int r = 0; r < kRing - 1; ++r) load(r, ring[r]);
        for (int i = 0; i < nb; i += kRing) {
#pragma unroll
            for (int r = 0; r < kRing; ++r) {
                load(i + r + kRing - 1, ring[(r + kRing - 1) % kRing]);
                if (r == 0 || i + r < nb) run(ring[r]);
            }
        }
        // ... then the tiles of pairs too long for the row stream, one
        // wavefront per pair
        for (int i = 0; i < nb; ++i) {
            const uint32_t e0 = (uint32_t)__builtin_amdgcn_readlane((int)r0, i);
            if ((e0 >> 30) == kBlkStream) continue;
            const uint32_t e1 = (uint32_t)__builtin_amdgcn_readlane((int)r1, i);
            window_pairs<T, 8>(a, win, (int)(e0 & kBlkRowMask), (int)(e1 & kBlkRowMask));
        }
    }
}

// Second pass: workgroup b reads block b's partials run by run (window w's
// run of pairs from first[b][w] fills slots pre[b][w]..pre[b][w+1]; the
// window of a slot comes from a map built in LDS; all of a lane's loads in
// one round) and places each in LDS in row order, so that each of the block's
// rows then adds its own contiguous partials (its windows in order, four
// interleaved sums; 0 for a row with no entries), rounds once and, fused,
// forms w = alpha*y + x.
// Threads per workgroup of the adding pass: one per row of a 1,024-row
// block, sixteen wavefronts (two workgroups per compute unit fit the LDS,
// so eight wavefronts per SIMD hide the pass's three dependent rounds of
// loads: 22.7 us on the 1M-row Zipf matrix against 23.7 us with 512
// threads and 27.1 us with 256).
constexpr int kXsumBS = 1024;

template <typename T, bool FUSED>
__global__ __launch_bounds__(kXsumBS) void k_xwin_sum(XsumArgs a)
{
    constexpr int RPT = (int)(kXwinMaxRb / kXsumBS);   // rows per thread at most
    __shared__ double stage[kXwinStage];     // the block's partials in row order
    __shared__ uint16_t wof[kXwinStage];     // window of each slot
    __shared__ int pre[kXwinMaxWin + 1];
    __shared__ int first[kXwinMaxWin];
    const int b = (int)blockIdx.x;
    const int t = (int)threadIdx.x;
    const int S = a.nwin;
    const int64_t r0 = (int64_t)b * a.rb;
    // the pair ranges of the thread's rows r0 + t + kXsumBS*q (clamped rows for
    // threads without one: no load here sits in a branch, so none is waited
    // for early), in flight during the staging
    int s[RPT], e[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t ic = min(r0 + t + kXsumBS * q, a.m - 1);
        s[q] = a.pos_ptr[ic];
        e[q] = a.pos_ptr[ic + 1];
    }
    const int base = a.pos_ptr[r0];
    const int *bpre = a.pre + (int64_t)b * (S + 1);
    const int *bfirst = a.first + (int64_t)b * S;
    for (int w = t; w <= S; w += kXsumBS) {
        pre[w] = bpre[w];
        if (w < S) first[w] = bfirst[w];
    }
    __syncthreads();
    const int total = pre[S];
    // every slot of the block in one round of loads (U per lane; slots
    // clamped to the last one, so the loads are issued unconditionally):
    // first the slots' places in row order, which need nothing else, then,
    // once the map of windows is built, the partials
    constexpr int U = (int)(kXwinStage / kXsumBS);
    static_assert(U * kXsumBS == kXwinStage, "staging area is a whole number of rounds");
    uint16_t place[U];
    if (total > 0) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            place[u] = __builtin_nontemporal_load(a.rowpos + base + min(u * kXsumBS + t, total - 1));
    }
    for (int w = t; w < S; w += kXsumBS)
        for (int j = pre[w]; j < pre[w + 1]; ++j) wof[j] = (uint16_t)w;
    __syncthreads();
    if (total > 0) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int jj = min(u * kXsumBS + t, total - 1);
            const int w = wof[jj];
            v[u] = __builtin_nontemporal_load(a.part + first[w] + (jj - pre[w]));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u * kXsumBS + t < total) stage[place[u]] = v[u];
    }
    __syncthreads();
    // each row's partials are contiguous: four interleaved sums (a fixed
    // order, so the result is reproducible)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = r0 + t + kXsumBS * q;
        if (t + kXsumBS * q >= a.rb || i >= a.m) break;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int k = s[q] - base;
        const int ke = e[q] - base;
        for (; k + 4 <= ke; k += 4) {
            a0 += stage[k];
            a1 += stage[k + 1];
            a2 += stage[k + 2];
            a3 += stage[k + 3];
        }
        if (k < ke) a0 += stage[k];
        if (k + 1 < ke) a1 += stage[k + 1];
        if (k + 2 < ke) a2 += stage[k + 2];
        const double acc = (a0 + a1) + (a2 + a3);
        const T yt = (T)acc;
        ((T *)a.y)[i] = yt;
        if constexpr (FUSED) ((T *)a.w)[i] = fma_t((T)a.alpha, yt, ((const T *)a.x)[i]);
    }
}

namespace {

template <typename T, int BS, int WB, int E>
hipError_t L_xwin(const XwinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_xwin<T, BS, WB, E>), dim3((unsigned)a.nchunk), dim3(BS), 0, s, a);
    return hipGetLastError();
}

#define XENTRY(BS, KIB, E) {BS, KIB, E, {L_xwin<float, BS, KIB * 1024, E>, L_xwin<double, BS, KIB * 1024, E>}}

// (threads per workgroup, window KiB, row-stream entries per wavefront):
// 128 KiB windows leave room for one workgroup per compute unit, 64 KiB
// windows for two.
const XwinEntry kXwin[] = {
    XENTRY(512, 128, 256),
    XENTRY(1024, 128, 128),
    XENTRY(768, 128, 256),   // 161,840 bytes of LDS: twelve wavefronts of 256-entry tiles
    XENTRY(256, 64, 256),
    XENTRY(512, 64, 256),
};

}  // namespace

const XwinEntry *xwin_table(int *count)
{
    *count = (int)(sizeof(kXwin) / sizeof(kXwin[0]));
    return kXwin;
}

hipError_t launch_xwin_sum(int dtype, bool fused, const XsumArgs &a, hipStream_t s)
{
    if (a.m <= 0) return hipSuccess;
    const unsigned g = (unsigned)((a.m + a.rb - 1) / a.rb);
    if (dtype == 1) {
        if (fused) hipLaunchKernelGGL((k_xwin_sum<double, true>), dim3(g), dim3(kXsumBS), 0, s, a);
        else hipLaunchKernelGGL((k_xwin_sum<double, false>), dim3(g), dim3(kXsumBS), 0, s, a);
    } else {
        if (fused) hipLaunchKernelGGL((k_xwin_sum<float, true>), dim3(g), dim3(kXsumBS), 0, s, a);
        else hipLaunchKernelGGL((k_xwin_sum<float, false>), dim3(g), dim3(kXsumBS), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace spk
