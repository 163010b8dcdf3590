// Instantiation helpers: one translation unit per (stencil, dtype) registers
// its naive kernel and its list of MWD (diamond width, cells per lane) kernels.
#pragma once
#include "mwd.hpp"
#include "naive.hpp"
#include "registry.hpp"

namespace girih {

template <class S, typename Real, int DW, int VX>
hipError_t launch_mwd(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((mwd_row_kernel<S, Real, DW, VX>), grid, block, 0, stream,
                       *static_cast<const MwdArgs<Real>*>(args));
    return hipGetLastError();
}

template <class S, typename Real>
hipError_t launch_naive(const void* args, dim3 grid, dim3 block, hipStream_t stream) {
    hipLaunchKernelGGL((naive_step_kernel<S, Real>), grid, block, 0, stream,
                       *static_cast<const NaiveArgs<Real>*>(args));
    return hipGetLastError();
}

template <class S, typename Real, int DW, int VX>
void add_mwd(std::vector<KernelEntry>& t, int st, int dt) {
    using K = MwdKernel<S, Real, DW, VX>;
    t.push_back(KernelEntry{st, dt, AL_MWD, DW, VX, K::NT, K::LDS_BYTES, K::XOWN_MAX,
                            reinterpret_cast<const void*>(&mwd_row_kernel<S, Real, DW, VX>),
                            &launch_mwd<S, Real, DW, VX>});
}

template <class S, typename Real>
void add_naive(std::vector<KernelEntry>& t, int st, int dt) {
    t.push_back(KernelEntry{st, dt, AL_NAIVE, 0, 0, 256, 0, 0,
                            reinterpret_cast<const void*>(&naive_step_kernel<S, Real>),
                            &launch_naive<S, Real>});
}

// Variants per radius and element size.  Each keeps its z-rings in registers
// (2R values per (row, level) cell and x cell), so the register file bounds
// diamond width times cells per lane.
template <class S, typename Real>
void add_family(std::vector<KernelEntry>& t, int st, int dt) {
    add_naive<S, Real>(t, st, dt);
    if constexpr (S::R == 1) {
        add_mwd<S, Real, 4, 2>(t, st, dt);
        add_mwd<S, Real, 4, 4>(t, st, dt);
        add_mwd<S, Real, 8, 1>(t, st, dt);
        add_mwd<S, Real, 8, 2>(t, st, dt);
        add_mwd<S, Real, 8, 4>(t, st, dt);
        add_mwd<S, Real, 12, 1>(t, st, dt);
        add_mwd<S, Real, 12, 2>(t, st, dt);
        add_mwd<S, Real, 16, 1>(t, st, dt);
        if constexpr (sizeof(Real) == 4) {
            add_mwd<S, Real, 12, 4>(t, st, dt);
            add_mwd<S, Real, 16, 2>(t, st, dt);
            add_mwd<S, Real, 16, 4>(t, st, dt);
        }
    } else {
        add_mwd<S, Real, 8, 1>(t, st, dt);
        add_mwd<S, Real, 8, 2>(t, st, dt);
        add_mwd<S, Real, 8, 4>(t, st, dt);
        add_mwd<S, Real, 16, 1>(t, st, dt);
        add_mwd<S, Real, 16, 2>(t, st, dt);
        add_mwd<S, Real, 24, 1>(t, st, dt);
        if constexpr (sizeof(Real) == 4) {
            add_mwd<S, Real, 16, 4>(t, st, dt);
            add_mwd<S, Real, 24, 2>(t, st, dt);
        }
    }
}

}  // namespace girih
