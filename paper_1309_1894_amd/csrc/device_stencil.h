// device_stencil.h -- row geometry of a constant-coefficient grid stencil,
// shared by the stencil SpMV and the conjugate-gradient SpMV+dot.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace spk {

// Grid neighbours of row r in ascending offset order (-N2*N3, -N3, -1, 0,
// +1, +N3, +N2*N3): clamped addresses and presence flags.
template <int DIM>
__device__ __forceinline__ void stencil_row(const StencilArgs &a, int r, int *at, bool *has)
{
    const uint32_t ur = (uint32_t)r;
    const uint32_t N3 = (uint32_t)a.N3, N2 = (uint32_t)a.N2;
    const uint32_t k = ur % N3;
    const uint32_t pencil = ur / N3;
    const uint32_t j = DIM >= 2 ? pencil % N2 : 0u;
    const uint32_t i = DIM >= 3 ? pencil / N2 : 0u;
    const int plane = a.N2 * a.N3, last = a.n - 1;
    has[0] = DIM >= 3 && i > 0;
    has[1] = DIM >= 2 && j > 0;
    has[2] = k > 0;
    has[3] = true;
    has[4] = k + 1 < N3;
    has[5] = DIM >= 2 && j + 1 < N2;
    has[6] = DIM >= 3 && i + 1 < (uint32_t)a.N1;
    at[0] = max(r - plane, 0);
    at[1] = max(r - a.N3, 0);
    at[2] = max(r - 1, 0);
    at[3] = r;
    at[4] = min(r + 1, last);
    at[5] = min(r + a.N3, last);
    at[6] = min(r + plane, last);
}

template <int DIM>
__device__ __forceinline__ constexpr bool stencil_slot(int q)
{
    return (q == 0 || q == 6) ? DIM >= 3 : (q == 1 || q == 5) ? DIM >= 2 : true;
}

}  // namespace spk
