// kernels_batch.hip -- one launch over many independent CSR instances.
//
// The host planner cuts every instance into tiles (row ranges) and gives
// each tile the kernel chosen for the instance's shape class: an LDS-staged
// row stream (mode 0) or G lanes per row (mode G).  The kernel either runs
// one workgroup per tile, or is persistent: a grid sized to fill the GPU
// pulls tiles from a queue head in device memory until the queue is empty.
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

template <typename T, int BS, int TILE>
__device__ __forceinline__ void run_tile(const BatchArgs<T> &a, int tile, double *sp, int *srp)
{
    const BatchTile td = a.tiles[tile];
    const int32_t *rp = td.rp;
    const int32_t *ci = td.ci;
    const T *val = (const T *)td.val;
    const T *x = a.x + td.vec_off;
    T *y = a.y + td.vec_off;
    T *w = a.w ? a.w + td.vec_off : nullptr;
    switch (td.mode) {
    case 0:  // entries of the tile fit the LDS tile (guaranteed by the planner)
        stream_rows<T, BS, TILE>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1, td.k0, td.k1, sp, srp);
        break;
    case 2: group_rows<T, BS, 2>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 4: group_rows<T, BS, 4>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 8: group_rows<T, BS, 8>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 16: group_rows<T, BS, 16>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    case 32: group_rows<T, BS, 32>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    default: group_rows<T, BS, 64>(rp, ci, val, x, y, w, a.alpha, td.r0, td.r1); break;
    }
}

template <typename T, int BS, int TILE>
__global__ __launch_bounds__(BS) void k_batch_grid(BatchArgs<T> a)
{
    __shared__ double sp[TILE];
    __shared__ int srp[kStreamRowsPerThread * BS + 1];
    run_tile<T, BS, TILE>(a, (int)blockIdx.x, sp, srp);
}

template <typename T, int BS, int TILE>
__global__ __launch_bounds__(BS) void k_batch_persistent(BatchArgs<T> a)
{
    __shared__ double sp[TILE];
    __shared__ int srp[kStreamRowsPerThread * BS + 1];
    __shared__ int s_tile;
    const int t = threadIdx.x;
    if (t == 0) s_tile = (int)atomicAdd(a.next, 1u);
    __syncthreads();
    int tile = s_tile;
    __syncthreads();
    while (tile < a.ntiles) {
        // the next index is claimed now and read after this tile, so the
        // atomic's latency hides behind the tile's own loads
        int claimed = 0;
        if (t == 0) claimed = (int)atomicAdd(a.next, 1u);
        run_tile<T, BS, TILE>(a, tile, sp, srp);
        if (t == 0) s_tile = claimed;
        __syncthreads();
        tile = s_tile;
        __syncthreads();
    }
    // Every workgroup has drawn past the end of the queue before it counts
    // itself done, so the last one may reset both counters.
    if (t == 0) {
        __threadfence();
        const uint32_t d = atomicAdd(a.done, 1u);
        if (d == gridDim.x - 1u) {
            atomicExch(a.next, 0u);
            atomicExch(a.done, 0u);
        }
    }
}

namespace {

template <typename T, int BS, int TILE>
int occ_batch()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_batch_persistent<T, BS, TILE>),
                                                     BS, 0) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

template <typename T, int BS, int TILE, bool P>
hipError_t L_batch(const void *p, dim3 g, hipStream_t s)
{
    if constexpr (P)
        hipLaunchKernelGGL((k_batch_persistent<T, BS, TILE>), g, dim3(BS), 0, s, *(const BatchArgs<T> *)p);
    else
        hipLaunchKernelGGL((k_batch_grid<T, BS, TILE>), g, dim3(BS), 0, s, *(const BatchArgs<T> *)p);
    return hipGetLastError();
}

#define BENTRY(BS, TILE) {BS, TILE, {{L_batch<float, BS, TILE, false>, L_batch<float, BS, TILE, true>}, \
                                     {L_batch<double, BS, TILE, false>, L_batch<double, BS, TILE, true>}}, \
                         {occ_batch<float, BS, TILE>, occ_batch<double, BS, TILE>}}

const BatchEntry kBatch[] = {
    BENTRY(256, 2048), BENTRY(256, 1024), BENTRY(256, 4096),
    BENTRY(128, 1024), BENTRY(128, 2048),
    BENTRY(512, 2048), BENTRY(512, 4096),
};

}  // namespace

const BatchEntry *batch_table(int *count)
{
    *count = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
    return kBatch;
}

}  // namespace spk
