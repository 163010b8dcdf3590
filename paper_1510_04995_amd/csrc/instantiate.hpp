// Instantiation helpers: one translation unit per (stencil, dtype) registers
// its naive kernel and its list of MWD (diamond width, cells per lane) kernels.
#pragma once
#include "mwd.hpp"
#include "naive.hpp"
#include "registry.hpp"

namespace girih {

template <class S, typename Real, int DW, int VX, int WX, int NSV, int NF, int SY>
hipError_t launch_mwd(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((mwd_row_kernel<S, Real, DW, VX, WX, NSV, NF, SY>), grid, block, 0, stream,
                       *static_cast<const MwdArgs<Real>*>(args));
    return hipGetLastError();
}

template <class S, typename Real>
hipError_t launch_naive(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_step_kernel<S, Real>), grid, block, 0, stream,
                       *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

template <class S, typename Real, int BY>
hipError_t launch_naive_tile(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_tile_kernel<S, Real, BY>), grid, block, 0, stream,
                       *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

template <class S, typename Real, int DW, int VX, int WX, int NF, int NSC, int SY>
hipError_t launch_sweep(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((mwd_sweep_kernel<S, Real, DW, VX, WX, NF, NSC, SY>), grid, block, 0, stream,
                       *static_cast<const MwdSweepArgs<Real>*>(args));
    return hipGetLastError();
}

// A diamond shape registers its full kernel and, where it is smaller, the
// kernel with H + 3 slots per wave: enough for the first diamond row (levels
// below H lie before t = 0) and for the last one (levels from H on lie at or
// after T).
// SWEEP: also compile the shape's dependency-driven whole-sweep kernel.
// SY: relaxed synchronisation within the tile (per-wave step counters
// instead of workgroup barriers).
template <class S, typename Real, int DW, int VX, int WX, int NF = 1, bool SWEEP = false, int SY = 0>
void add_mwd(std::vector<KernelEntry>& t, int st, int dt) {
    using K = MwdKernel<S, Real, DW, VX, WX, NF>;
    constexpr int H = K::H, L = K::L;
    constexpr int NSC = H + 3 < L + 2 ? H + 3 : 0;
    constexpr int LDS = K::LDS_BYTES + (SY ? 128 : 0);
    t.push_back(KernelEntry{st, dt, AL_MWD, DW, VX, WX, K::NT, LDS, K::XOWN_MAX, 0, 0, NF,
                            reinterpret_cast<const void*>(&mwd_row_kernel<S, Real, DW, VX, WX, 0, NF, SY>),
                            &launch_mwd<S, Real, DW, VX, WX, 0, NF, SY>});
    t.back().sync = SY;
    if constexpr (SWEEP) {
        t.back().sweep_func = reinterpret_cast<const void*>(&mwd_sweep_kernel<S, Real, DW, VX, WX, NF, NSC, SY>);
        t.back().launch_sweep = &launch_sweep<S, Real, DW, VX, WX, NF, NSC, SY>;
    }
    if constexpr (H + 3 < L + 2) {
        t.push_back(KernelEntry{st, dt, AL_MWD, DW, VX, WX, K::NT, LDS, K::XOWN_MAX, H + 3, 0, NF,
                                reinterpret_cast<const void*>(&mwd_row_kernel<S, Real, DW, VX, WX, H + 3, NF, SY>),
                                &launch_mwd<S, Real, DW, VX, WX, H + 3, NF, SY>});
        t.back().sync = SY;
    }
}

template <class S, typename Real, int BY>
void add_naive_tile(std::vector<KernelEntry>& t, int st, int dt) {
    constexpr int R = S::R;
    t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, 0, 0, 64 * BY, (BY + 2 * R) * (64 + 2 * R) * (int)sizeof(Real), 0,
                            0, 1, 0, reinterpret_cast<const void*>(&naive_tile_kernel<S, Real, BY>),
                            &launch_naive_tile<S, Real, BY>});
}

template <typename Real>
hipError_t launch_naive_box(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_box_kernel<Real>), grid, block, 0, stream, *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

template <typename Real, int KY>
hipError_t launch_naive_box_cols(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_box_cols_kernel<Real, KY>), grid, block, 0, stream,
                       *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

// register columns: blocks of 64 x W threads, KY rows per lane (vx = KY)
template <typename Real, int KY>
void add_box_cols(std::vector<KernelEntry>& t, int st, int dt) {
    for (int w : {2, 4})
        t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, KY, 0, 64 * w, 0, 0, 0, 1, 0,
                                reinterpret_cast<const void*>(&naive_box_cols_kernel<Real, KY>),
                                &launch_naive_box_cols<Real, KY>});
}

// The 27-point box stencil: the naive sweep with cached neighbours (variant
// 0) or register columns (variant 1), and the blocked sweep with its
// three-plane stage rows (one CU holds them at Dw = 8 in FP64, 159 of 160
// KiB, and up to Dw = 12 in FP32).
template <typename Real>
void add_box_family(std::vector<KernelEntry>& t, int st, int dt) {
    t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, 0, 0, 256, 0, 0, 0, 0, 0,
                            reinterpret_cast<const void*>(&naive_box_kernel<Real>), &launch_naive_box<Real>});
    add_box_cols<Real, 2>(t, st, dt);
    add_box_cols<Real, 4>(t, st, dt);
    add_box_cols<Real, 8>(t, st, dt);
    add_mwd<Stencil27B, Real, 8, 1, 2, 1, false, 0>(t, st, dt);
    if constexpr (sizeof(Real) == 4) add_mwd<Stencil27B, Real, 12, 1, 2, 1, false, 0>(t, st, dt);
}

template <class S, typename Real, int KY>
hipError_t launch_naive_star_cols(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_star_cols_kernel<S, Real, KY>), grid, block, 0, stream,
                       *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

// register columns (variant 2): blocks of 64 x W threads, KY rows per lane (vx = KY)
template <class S, typename Real, int KY>
void add_star_cols(std::vector<KernelEntry>& t, int st, int dt) {
    for (int w : {2, 4})
        t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, KY, 0, 64 * w, 0, 0, 0, 2, 0,
                                reinterpret_cast<const void*>(&naive_star_cols_kernel<S, Real, KY>),
                                &launch_naive_star_cols<S, Real, KY>});
}

template <class S, typename Real>
void add_naive(std::vector<KernelEntry>& t, int st, int dt) {
    t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, 0, 0, 256, 0, 0, 0, 0, 0,
                            reinterpret_cast<const void*>(&naive_step_kernel<S, Real>),
                            &launch_naive<S, Real>});
    add_naive_tile<S, Real, 4>(t, st, dt);
    add_naive_tile<S, Real, 8>(t, st, dt);
    add_naive_tile<S, Real, 16>(t, st, dt);
    if constexpr (S::NCOEF == 0 && !S::LEAPFROG) {
        add_star_cols<S, Real, 2>(t, st, dt);
        add_star_cols<S, Real, 4>(t, st, dt);
        add_star_cols<S, Real, 8>(t, st, dt);
    }
}

// Variants per radius and element size.  Each keeps its z-rings in registers
// (2R values per (row, level) cell and x cell), so the register file bounds
// diamond width times cells per lane; only shapes whose wavefront loops run
// without register spills are listed.
template <class S, typename Real>
void add_family(std::vector<KernelEntry>& t, int st, int dt) {
    add_naive<S, Real>(t, st, dt);
    constexpr bool F64 = sizeof(Real) == 8;
    // The second-order-in-time stencil: a level also reads the level two
    // below at its own cell (from the ring two slots back, or for a row's
    // first level from HBM) and its C array like a coefficient array.
    if constexpr (S::LEAPFROG) {
        add_mwd<S, Real, 16, 1, 1, 1, F64>(t, st, dt);
        add_mwd<S, Real, 8, 1, 2>(t, st, dt);
        if constexpr (!F64) add_mwd<S, Real, 16, 1, 1, 2>(t, st, dt);
    } else if constexpr (S::NCOEF > 0 && S::R == 1) {
        // Variable coefficients: every slot also holds the byte offset of its
        // coefficient row, so fewer register slots fit than for the constant
        // stencil (Dw = 12 spills in FP64).
        // (shapes marked true also get the dependency-driven whole-sweep kernel)
        add_mwd<S, Real, 8, 1, 2, 1, F64>(t, st, dt);
        add_mwd<S, Real, 8, 2, 1>(t, st, dt);
        add_mwd<S, Real, 8, 1, 2, 2>(t, st, dt);
        if constexpr (F64) {
            add_mwd<S, Real, 8, 1, 3>(t, st, dt);
        } else {
            add_mwd<S, Real, 8, 1, 4>(t, st, dt);
            add_mwd<S, Real, 12, 1, 2, 1, true>(t, st, dt);
            add_mwd<S, Real, 12, 2, 1>(t, st, dt);
            add_mwd<S, Real, 16, 1, 1>(t, st, dt);
        }
    } else if constexpr (S::NCOEF > 0) {
        add_mwd<S, Real, 8, 1, 2>(t, st, dt);
        add_mwd<S, Real, 8, 2, 1>(t, st, dt);
        if constexpr (F64) {
            add_mwd<S, Real, 8, 1, 1>(t, st, dt);
        } else {
            add_mwd<S, Real, 16, 1, 1>(t, st, dt);
        }
    } else if constexpr (S::R == 1) {
        // (diamond width, cells per lane, waves along x)
        add_mwd<S, Real, 4, 2, 2>(t, st, dt);
        add_mwd<S, Real, 8, 1, 2, 1, true>(t, st, dt);
        add_mwd<S, Real, 8, 1, 3>(t, st, dt);
        add_mwd<S, Real, 8, 2, 1>(t, st, dt);
        add_mwd<S, Real, 8, 2, 2>(t, st, dt);
        add_mwd<S, Real, 12, 1, 2, 1, true>(t, st, dt);
        add_mwd<S, Real, 16, 1, 1>(t, st, dt);
        // relaxed synchronisation within the tile
        add_mwd<S, Real, 12, 1, 2, 1, true, 1>(t, st, dt);
        // wavefront depth 2 (two planes per step): twice the stage rows and
        // ring registers of depth 1
        add_mwd<S, Real, 8, 1, 2, 2>(t, st, dt);
        if constexpr (!F64) {
            add_mwd<S, Real, 8, 1, 4>(t, st, dt);
            add_mwd<S, Real, 12, 2, 1>(t, st, dt);
            add_mwd<S, Real, 16, 2, 1>(t, st, dt);
            add_mwd<S, Real, 12, 1, 2, 2, true>(t, st, dt);
            add_mwd<S, Real, 16, 1, 1, 2>(t, st, dt);
            add_mwd<S, Real, 12, 1, 2, 2, true, 1>(t, st, dt);
        }
    } else {
        add_mwd<S, Real, 8, 1, 2>(t, st, dt);
        add_mwd<S, Real, 8, 2, 1>(t, st, dt);
        add_mwd<S, Real, 16, 1, 1, 1, F64>(t, st, dt);
        if constexpr (!F64) {
            add_mwd<S, Real, 8, 1, 4>(t, st, dt);
            add_mwd<S, Real, 8, 2, 2>(t, st, dt);
            add_mwd<S, Real, 16, 2, 1, 1, true>(t, st, dt);
            add_mwd<S, Real, 24, 1, 1>(t, st, dt);
            add_mwd<S, Real, 16, 1, 1, 2, true>(t, st, dt);
        }
    }
}

}  // namespace girih
