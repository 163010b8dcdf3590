// Naive two-buffer Jacobi step (paper, Section "Background / Cache blocking":
// every step sweeps the whole domain, no reuse across steps).  This is the
// comparator of the blocked sweep and executes the same per-point code
// (stencils.hpp) in the same operand order.
//
// Launch shape: a 2-D tile of (BX lanes along x) x (BY waves along y) marches
// along z over z_chunk planes.  Each lane keeps the 2R+1 z-window of its
// column in registers (each plane is read from memory once per lane); x and y
// neighbours of the centre plane come from the same coalesced rows through
// the L1/L2 caches.  x is the fastest index, so every access is a contiguous
// x-row of the wave.
#pragma once
#include "stencils.hpp"

namespace girih {

template <typename Real>
struct NaiveArgs {
    GridDesc g;
    const Real* V;    // time level t
    Real* U;          // time level t+1
    CoefArgs<Real> coef;
    int32_t z_chunk;
};

template <class S, typename Real>
__global__ void __launch_bounds__(256)
naive_step_kernel(NaiveArgs<Real> a) {
    constexpr int R = S::R;
    const GridDesc& g = a.g;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t y = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const int64_t z0 = (int64_t)blockIdx.z * a.z_chunk;
    int64_t z1 = z0 + a.z_chunk;
    if (z1 > g.nz) z1 = g.nz;
    if (z0 >= z1) return;
    const int64_t plane = g.plane();
    const int64_t px = g.pitch_x;
    const Real* __restrict__ V = a.V;
    Real* __restrict__ U = a.U;
    // z-window: w[0..2R] = planes z-R..z+R of this column
    Real w[2 * R + 1];
    int64_t p = g.idx(z0, y, x);
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) w[m] = V[p + (m - R) * plane];
    for (int64_t z = z0; z < z1; ++z, p += plane) {
        w[2 * R] = V[p + R * plane];
        Nbhd<Real, R> n;
        n.c = w[R];
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            n.xp[r - 1] = V[p + r];
            n.xm[r - 1] = V[p - r];
            n.yp[r - 1] = V[p + r * px];
            n.ym[r - 1] = V[p - r * px];
            n.zp[r - 1] = w[R + r];
            n.zm[r - 1] = w[R - r];
        }
        Real cf[S::NCOEF > 0 ? S::NCOEF : 1];
#pragma unroll
        for (int m = 0; m < S::NCOEF; ++m) cf[m] = a.coef.arr[m][p];
        U[p] = S::apply(n, a.coef.k, cf);
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) w[m] = w[m + 1];
    }
}

}  // namespace girih
