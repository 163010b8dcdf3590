// Table of compiled kernels.  Every instantiated kernel registers one entry;
// the planner and the tuner pick from this table, so the tuning space is
// exactly what was compiled.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

namespace girih {

enum StencilId { ST_7C = 0, ST_7V = 1, ST_25C = 2, ST_25V = 3, ST_25L = 4, ST_27B = 5 };
enum DtypeId { DT_F64 = 0, DT_F32 = 1 };
enum AlgoId { AL_NAIVE = 0, AL_MWD = 1 };

using LaunchFn = hipError_t (*)(const void* args, dim3 grid, dim3 block, hipStream_t stream);

struct KernelEntry {
    int stencil;
    int dtype;
    int algo;
    int dw;          // MWD diamond width
    int vx;          // MWD x cells per lane
    int wx;          // MWD waves along x per row pair (a row holds 64*vx*wx cells)
    int nthreads;    // MWD workgroup size
    int lds_bytes;   // static LDS per workgroup
    int xown_max;    // MWD: largest owned x tile
    int ns;          // MWD: register slots per wave (0: all L + 2; fewer: rows clipped by the run's time bounds)
    int variant;     // naive: 0 = neighbours through the caches, 1 = plane tiles in LDS (nthreads = 64 x rows)
    int nf;          // MWD: wavefront depth (planes per wavefront step)
    const void* func;
    LaunchFn launch;
    // MWD, full slot count: the dependency-driven whole-sweep kernel of the
    // shape (one launch, persistent workgroups), or null where none is compiled
    const void* sweep_func = nullptr;
    LaunchFn launch_sweep = nullptr;
    // MWD: 0 = workgroup barriers between the phases of a wavefront step,
    // 1 = relaxed synchronisation (per-wave step counters in LDS)
    int sync = 0;
};

void register_kernels_7c_f64(std::vector<KernelEntry>&);
void register_kernels_7c_f32(std::vector<KernelEntry>&);
void register_kernels_7v_f64(std::vector<KernelEntry>&);
void register_kernels_7v_f32(std::vector<KernelEntry>&);
void register_kernels_25c_f64(std::vector<KernelEntry>&);
void register_kernels_25c_f32(std::vector<KernelEntry>&);
void register_kernels_25v_f64(std::vector<KernelEntry>&);
void register_kernels_25v_f32(std::vector<KernelEntry>&);
void register_kernels_25l_f64(std::vector<KernelEntry>&);
void register_kernels_25l_f32(std::vector<KernelEntry>&);
void register_kernels_27b_f64(std::vector<KernelEntry>&);
void register_kernels_27b_f32(std::vector<KernelEntry>&);

const std::vector<KernelEntry>& kernel_table();

// utility kernels (util.hip)
hipError_t launch_copy_halo(const void* src, void* dst, int elem_bytes, int64_t nx, int64_t ny, int64_t nz,
                            int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s);
hipError_t launch_zero_halo_flag(const void* src, int* flag, int elem_bytes, int64_t nx, int64_t ny, int64_t nz,
                                 int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s);
hipError_t error_norms(const void* a, int dta, const void* b, int dtb, int64_t nx, int64_t ny, int64_t nz,
                       int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s, double out[4]);

}  // namespace girih
