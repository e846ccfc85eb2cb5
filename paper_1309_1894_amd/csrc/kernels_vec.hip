// kernels_vec.hip -- WAXPY/AXPY and dot kernels for gfx950.
//
// Both are pure HBM streams (WAXPY moves 3 words per element for 2 flops,
// dot 2 words), so the variants differ only in how the stream is cut:
// threads per workgroup (BS), elements per lane access (VEC, up to 16-byte
// global_load_dwordx4), independent accesses in flight per lane (UNR) and
// the grid (one pass, or a grid-stride loop over a fixed number of
// workgroups per CU).  Section 3 of the paper lists exactly these knobs
// (threads per block, blocks per grid, unroll) as the search space.
#include "device_common.h"
#include "kernels.h"

namespace spk {

// Streams are touched once: loads and stores carry the non-temporal hint.
template <typename T, int VEC>
struct ntvec;
template <typename T>
struct ntvec<T, 1> {
    typedef T type;
};
template <>
struct ntvec<double, 2> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct ntvec<float, 2> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct ntvec<float, 4> {
    typedef float type __attribute__((ext_vector_type(4)));
};

template <typename T, int VEC>
__device__ __forceinline__ vec_t<T, VEC> nt_load(const T *p)
{
    using N = typename ntvec<T, VEC>::type;
    const N v = __builtin_nontemporal_load(reinterpret_cast<const N *>(p));
    vec_t<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = v;
    } else {
#pragma unroll
        for (int j = 0; j < VEC; ++j) r.v[j] = v[j];
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void nt_store(T *p, const vec_t<T, VEC> &r)
{
    using N = typename ntvec<T, VEC>::type;
    N v;
    if constexpr (VEC == 1) {
        v = r.v[0];
    } else {
#pragma unroll
        for (int j = 0; j < VEC; ++j) v[j] = r.v[j];
    }
    __builtin_nontemporal_store(v, reinterpret_cast<N *>(p));
}

// w_i = alpha*x_i + y_i.  w may be x or y (each element is read before it
// is written by the same lane, and no lane touches another's elements).
template <typename T, int BS, int VEC, int UNR>
__global__ __launch_bounds__(BS) void k_waxpy(int64_t n, T alpha, const T *x, const T *y, T *w)
{
    using V = vec_t<T, VEC>;
    constexpr int64_t PER = (int64_t)BS * VEC * UNR;
    const int t = threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * PER;
    for (int64_t base = (int64_t)blockIdx.x * PER; base < n; base += stride) {
        if (base + PER <= n) {
            V xv[UNR], yv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t i = base + ((int64_t)u * BS + t) * VEC;
                xv[u] = nt_load<T, VEC>(x + i);
                yv[u] = nt_load<T, VEC>(y + i);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t i = base + ((int64_t)u * BS + t) * VEC;
                V r;
#pragma unroll
                for (int j = 0; j < VEC; ++j) r.v[j] = fma_t(alpha, xv[u].v[j], yv[u].v[j]);
                nt_store<T, VEC>(w + i, r);
            }
        } else {
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int64_t i = base + ((int64_t)u * BS + t) * VEC + j;
                    if (i < n) w[i] = fma_t(alpha, x[i], y[i]);
                }
            }
        }
    }
}

// d = sum_i x_i*y_i in FP64.  Each lane keeps UNR running FMA chains over a
// fixed set of elements, the workgroup reduces them (DPP within waves, LDS
// across waves) into partial[blockIdx.x].  Small grids finish in the same
// launch: the last workgroup to finish (ticket) adds the partials in index
// order.  Without a ticket the kernel only leaves the partials and
// k_dot_final adds them in the same order in a second launch: each
// workgroup would otherwise publish its partial with a device-scope
// release, which writes back its XCD's L2 and serialises there (tens of
// microseconds at a thousand workgroups).  The order of every addition
// depends only on (n, variant), so results are reproducible bit for bit.
template <typename T, int BS, int VEC, int UNR>
__global__ __launch_bounds__(BS) void k_dot(int64_t n, const T *x, const T *y, double *partial,
                                            uint32_t *ticket, double *out)
{
    using V = vec_t<T, VEC>;
    constexpr int64_t PER = (int64_t)BS * VEC * UNR;
    __shared__ double red[BS / kWave > 0 ? BS / kWave : 1];
    __shared__ int is_last;
    const int t = threadIdx.x;
    double acc[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) acc[u] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * PER;
    for (int64_t base = (int64_t)blockIdx.x * PER; base < n; base += stride) {
        if (base + PER <= n) {
            V xv[UNR], yv[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t i = base + ((int64_t)u * BS + t) * VEC;
                xv[u] = nt_load<T, VEC>(x + i);
                yv[u] = nt_load<T, VEC>(y + i);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    acc[u] = fma_t((double)xv[u].v[j], (double)yv[u].v[j], acc[u]);
        } else {
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int64_t i = base + ((int64_t)u * BS + t) * VEC + j;
                    if (i < n) acc[u] = fma_t((double)x[i], (double)y[i], acc[u]);
                }
        }
    }
    double s = acc[0];
#pragma unroll
    for (int u = 1; u < UNR; ++u) s += acc[u];
    s = block_sum<BS>(s, red);
    if (!ticket) {
        if (t == 0) partial[blockIdx.x] = s;
        return;
    }
    if (t == 0) {
        partial[blockIdx.x] = s;
        __threadfence();
        const uint32_t prev = atomicAdd(ticket, 1u);
        is_last = (prev == gridDim.x - 1u);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        double a = 0.0;
        for (int64_t i = t; i < (int64_t)gridDim.x; i += BS) a += partial[i];
        a = block_sum<BS>(a, red);
        if (t == 0) {
            *out = a;
            *ticket = 0u;
        }
    }
}

// *out = sum of partial[0, count): the partials in index-strided order
// per lane, then the workgroup tree.
template <int BS>
__global__ __launch_bounds__(BS) void k_dot_final(const double *partial, int64_t count, double *out)
{
    __shared__ double red[BS / kWave];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += BS) a += partial[i];
    a = block_sum<BS>(a, red);
    if (threadIdx.x == 0) *out = a;
}

hipError_t launch_dot_final(const double *partial, int64_t count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_final<1024>, dim3(1), dim3(1024), 0, s, partial, count, out);
    return hipGetLastError();
}

namespace {

template <typename T, int BS, int VEC, int UNR>
hipError_t launch_waxpy(const VecLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL((k_waxpy<T, BS, VEC, UNR>), dim3((unsigned)L.grid), dim3(BS), 0, s, L.n,
                       (T)L.alpha, (const T *)L.x, (const T *)L.y, (T *)L.w);
    return hipGetLastError();
}

template <typename T, int BS, int VEC, int UNR>
hipError_t launch_dot(const VecLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL((k_dot<T, BS, VEC, UNR>), dim3((unsigned)L.grid), dim3(BS), 0, s, L.n,
                       (const T *)L.x, (const T *)L.y, L.partial, L.ticket, L.out);
    return hipGetLastError();
}

// FP32 uses VEC in {1,2,4}, FP64 in {1,2}: at most 16 bytes per access.
#define SPK_VEC_ROW(KIND, BS, VEC, UNR)                                              \
    {BS, VEC, UNR,                                                                   \
     {launch_##KIND<float, BS, VEC, UNR>,                                            \
      (VEC * 8 <= 16) ? (VecFn)launch_##KIND<double, BS, (VEC <= 2 ? VEC : 2), UNR> : nullptr}}

#define SPK_VEC_UNR(KIND, BS, VEC) \
    SPK_VEC_ROW(KIND, BS, VEC, 1), SPK_VEC_ROW(KIND, BS, VEC, 2), SPK_VEC_ROW(KIND, BS, VEC, 4), SPK_VEC_ROW(KIND, BS, VEC, 8)

#define SPK_VEC_VEC(KIND, BS) SPK_VEC_UNR(KIND, BS, 1), SPK_VEC_UNR(KIND, BS, 2), SPK_VEC_UNR(KIND, BS, 4)

const VecEntry kWaxpy[] = {
    SPK_VEC_VEC(waxpy, 64), SPK_VEC_VEC(waxpy, 128), SPK_VEC_VEC(waxpy, 256),
    SPK_VEC_VEC(waxpy, 512), SPK_VEC_VEC(waxpy, 1024),
};

const VecEntry kDot[] = {
    SPK_VEC_VEC(dot, 128), SPK_VEC_VEC(dot, 256), SPK_VEC_VEC(dot, 512), SPK_VEC_VEC(dot, 1024),
};

#undef SPK_VEC_VEC
#undef SPK_VEC_UNR
#undef SPK_VEC_ROW

}  // namespace

const VecEntry *waxpy_table(int *count)
{
    *count = (int)(sizeof(kWaxpy) / sizeof(kWaxpy[0]));
    return kWaxpy;
}

const VecEntry *dot_table(int *count)
{
    *count = (int)(sizeof(kDot) / sizeof(kDot[0]));
    return kDot;
}

}  // namespace spk
