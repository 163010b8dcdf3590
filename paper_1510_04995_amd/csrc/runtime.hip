// Host runtime of the library: plans, the diamond-row launcher, the tuner and
// the C ABI declared in include/girih.h.
//
// Runtime (paper, Section "Runtime system"): the paper's runtime hands ready
// tiles to thread groups through a FIFO queue; a row of diamonds has no
// internal dependencies and each row depends only on the previous one, so on
// the GPU one kernel launch per row is the queue: the hardware dispatcher
// hands the row's workgroups to compute units as they free up, and stream
// order is the row barrier.
//
// Tuner (paper, Section "Auto-tuning"): it allocates its own arrays, times
// candidates on back-to-back runs of the problem's own T-step schedule, their
// number doubled until two consecutive measurements agree, and searches
// either every feasible candidate or, per thread shape, by hill climbing over
// the diamond width, the wavefront depth and the x tile.  The on-chip
// capacity bound (the paper prunes with its cache block size model and the
// user's cache size) is exact here: only compiled kernels whose LDS and
// registers fit exist in the table, and a user budget below the CU's LDS
// prunes further (girih_set_lds_budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "../../include/girih.h"
#include "registry.hpp"
#include "stencils.hpp"
#include "naive.hpp"
#include "mwd.hpp"

using namespace girih;

namespace girih {

const std::vector<KernelEntry>& kernel_table() {
    static const std::vector<KernelEntry> table = [] {
        std::vector<KernelEntry> t;
        register_kernels_7c_f64(t);
        register_kernels_7c_f32(t);
        register_kernels_7v_f64(t);
        register_kernels_7v_f32(t);
        register_kernels_25c_f64(t);
        register_kernels_25c_f32(t);
        register_kernels_25v_f64(t);
        register_kernels_25v_f32(t);
        register_kernels_25l_f64(t);
        register_kernels_25l_f32(t);
        register_kernels_27b_f64(t);
        register_kernels_27b_f32(t);
        return t;
    }();
    return table;
}

}  // namespace girih

namespace {

constexpr int kNStencils = 6;
constexpr int kRadius[kNStencils] = {1, 1, 4, 4, 4, 1};
constexpr int kNCoef[kNStencils] = {0, 7, 0, 13, 1, 0};
constexpr int kNConst[kNStencils] = {2, 0, 5, 0, 5, 4};
// domain-sized arrays a naive step streams: V and U, the coefficient arrays,
// and for the second-order-in-time stencil U's old value read before it is
// overwritten (U is read and written)
constexpr int kStreams[kNStencils] = {2, 9, 2, 15, 4, 2};

struct Tuning {
    std::vector<girih_params> model_cands;
    std::vector<girih_tune_record> log;
};

}  // namespace

struct girih_plan_s {
    int stencil = 0, dtype = 0, algo = 0;
    girih_grid grid{};
    double consts[5] = {0, 0, 0, 0, 0};
    girih_params params{};
    const KernelEntry* kern = nullptr;   // MWD variant or naive kernel
    int R = 1;
    int64_t x_own = 0, n_xchunks = 0;
    void* work[2] = {nullptr, nullptr};  // the MWD pair beside the caller's (allocated on the first run)
    int* halo_flag = nullptr;            // device int: input halo is all zero
    size_t work_bytes = 0;
    int work_device = -1;
    // dependency-driven schedule (variant 1): queue counters, error word and
    // completion marks on the device, and the marks' base for the next run
    uint32_t* sched = nullptr;
    int64_t sched_words = 0;
    int sched_device = -1;
    uint32_t sched_base = 1;
    uint32_t spin_limit = 1u << 20;
    int64_t lds_budget = 0;   // tuner's on-chip budget (0: the CU's)
    // error word of the last run's bounded waits (null: the run had none)
    uint32_t* err_word = nullptr;
    Tuning tuning;
    // per-launch timing of the sweep kernels (girih_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> events;   // pairs: before / after each sweep launch
    int n_timed = 0;
};

namespace {

size_t elem_bytes(int dtype) { return dtype == GIRIH_F64 ? 8 : 4; }

size_t grid_bytes(const girih_plan_s* p) {
    return (size_t)(p->grid.nz + 2 * p->grid.halo) * (size_t)p->grid.pitch_y * (size_t)p->grid.pitch_x *
           elem_bytes(p->dtype);
}

const KernelEntry* find_mwd(int st, int dt, int dw, int vx, int wx, int nf, int sync) {
    for (const auto& e : kernel_table())
        if (e.algo == AL_MWD && e.stencil == st && e.dtype == dt && e.dw == dw && e.vx == vx && e.wx == wx &&
            e.nf == nf && e.sync == sync && e.ns == 0)
            return &e;
    return nullptr;
}

// Register slots a wave of the diamond-row kernel needs in the row with time
// centre t_c of a T-step run: per wave, row A's input level and computed
// levels, then row B's (one slot for a row without levels).  Rows are paired
// as the kernel pairs them (half-distance block b with H-1-b); levels are
// clipped by the run's time bounds only, which bounds the kernel's count,
// where rows outside the grid hold one slot.
int mwd_slots_needed(int R, int dw, int64_t t_c, int64_t T) {
    const int H = dw / (2 * R), L = 2 * H;
    auto slots = [&](int d) {
        const int b = d / R;
        int64_t lo = b + 1, hi = L - 1 - b;
        lo = std::max<int64_t>(lo, H - t_c);
        hi = std::min<int64_t>(hi, T - 1 + H - t_c);
        return lo <= hi ? (int)(hi - lo + 2) : 1;
    };
    int need = 0;
    for (int d = 0; d < dw / 2; ++d) {
        const int b = d / R, e = d % R, b2 = H - 1 - b;
        const int pd = b2 != b ? b2 * R + e : b * R + (e ^ 1);
        if (d < pd) need = std::max(need, slots(d) + slots(pd));
    }
    return need;
}

// The kernel of a plan's diamond shape with the fewest slots that still hold
// `need`: the full kernel unless a clipped-row kernel suffices.
const KernelEntry* mwd_kernel_for(const KernelEntry* full, int need) {
    const KernelEntry* best = full;
    for (const auto& e : kernel_table())
        if (e.algo == AL_MWD && e.stencil == full->stencil && e.dtype == full->dtype && e.dw == full->dw &&
            e.vx == full->vx && e.wx == full->wx && e.nf == full->nf && e.sync == full->sync && e.ns > 0 &&
            e.ns >= need &&
            (best->ns == 0 || e.ns < best->ns))
            best = &e;
    return best;
}

// Naive kernel: variant 0 takes any block shape; variant 1 (plane tiles in
// LDS) exists for blocks of 64 x `rows` threads.
// For the box stencil variant 1 is register columns, for blocks of 64 x
// `rows` threads holding `cells` y rows per lane.
const KernelEntry* find_naive(int st, int dt, int variant, int rows, int cells) {
    for (const auto& e : kernel_table())
        if (e.algo == AL_NAIVE && e.stencil == st && e.dtype == dt && e.variant == variant &&
            (variant == 0 || e.nthreads == 64 * rows) && (e.vx == 0 || e.vx == cells))
            return &e;
    return nullptr;
}

// Default MWD shape per radius and element size (diamond width, cells per
// lane, waves along x); the tuner replaces it per problem.
void default_mwd(int stencil, int R, int dtype, int& dw, int& vx, int& wx, int& nf, int& var) {
    nf = 1;
    var = 0;
    // the dependency-driven schedule where it measured faster than row
    // launches with the default shape: 25-point constant FP64 (429 tiles a
    // row on 512^3, two rounds: +2 %) and 7-point variable FP64 (+4 %)
    if (dtype == GIRIH_F64 && (stencil == GIRIH_25PT_CONST || stencil == GIRIH_7PT_VAR)) var = 1;
    if (stencil == GIRIH_27PT_BOX) {
        // the widest box diamond whose three-plane stage fits one CU: 8 in
        // FP64, 12 in FP32 (twice the FP32 rate of Dw = 8 on 512^3, where its
        // workgroups fit the CUs in one round)
        dw = dtype == GIRIH_F32 ? 12 : 8;
        vx = 1;
        wx = 2;
    } else if (stencil == GIRIH_25PT_LEAPFROG) {
        // the widest radius-4 diamond that fits (Dw = 8 moves more bytes than
        // the naive sweep); FP32: two planes per wavefront step (measured
        // 32 % faster on 512^3)
        dw = 16;
        vx = 1;
        wx = 1;
        if (dtype == GIRIH_F32) nf = 2;
    } else if (kNCoef[stencil] > 0) {
        // variable coefficients: the per-slot coefficient offsets take the
        // registers a wider diamond would need (7-point FP32: Dw = 12 fits,
        // but measured 6 % slower than Dw = 8 on 256 x 512 x 1024)
        dw = dtype == GIRIH_F32 && R != 1 ? 16 : 8;
        vx = 1;
        wx = R == 1 || dtype == GIRIH_F64 ? 2 : 1;
    } else if (R == 1) {
        dw = 12;
        vx = 1;
        wx = 2;
        // FP32: two planes per wavefront step (measured 8 % faster on 512^3)
        if (dtype == GIRIH_F32) nf = 2;
    } else {
        // FP32 halves the z-ring registers: two cells per lane fit
        dw = 16;
        vx = dtype == GIRIH_F32 ? 2 : 1;
        wx = 1;
    }
}

// Default owned x tile: as many x chunks as keep one diamond row's
// workgroups within one round on the device's CUs (one workgroup per CU),
// but never a tile wider than the kernel holds nor narrower than half of
// that (the redundant x-halo grows as the tile shrinks).  More chunks in the
// same round spread a row's HBM traffic over more CUs.
int64_t default_x_tile(const girih_plan_s* p, const KernelEntry* k, int dw) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0) {
        (void)hipGetLastError();
        n_cu = 256;   // MI355X
    }
    const int64_t nx = p->grid.nx;
    const int64_t n_diamonds = (p->grid.ny + dw / 2 + dw - 1) / dw;   // the larger of the two row offsets
    const int64_t c_min = (nx + k->xown_max - 1) / k->xown_max;
    const int64_t c_max = std::max<int64_t>(1, n_cu / std::max<int64_t>(1, n_diamonds));
    const int64_t c_half = (nx + k->xown_max / 2 - 1) / std::max(1, k->xown_max / 2);
    const int64_t c = std::max(c_min, std::min({c_max, c_half, nx}));
    return (nx + c - 1) / c;
}

// Resolve and validate parameters; fills derived fields of the plan.
int resolve(girih_plan_s* p, const girih_params* in) {
    girih_params q{};
    if (in) q = *in;
    const int R = p->R;
    if (p->algo == GIRIH_MWD) {
        int dw = q.diamond_width, vx = q.cells_per_lane, wx = q.threads_x ? q.threads_x / 64 : 0;
        int ddw, dvx, dwx, dnf, dvar;
        default_mwd(p->stencil, R, p->dtype, ddw, dvx, dwx, dnf, dvar);
        if (q.threads_x < 0 || q.threads_x % 64 || vx < 0) return GIRIH_E_INVALID;
        if (dw == 0) dw = ddw;
        if (vx == 0 && wx == 0) { vx = dvx; wx = dwx; }
        if (vx == 0) vx = 1;
        if (wx == 0) wx = 1;
        if (dw <= 0 || dw % (2 * R) || (R == 1 && dw % 4)) return GIRIH_E_INVALID;
        // the default depth goes with the default shape only
        const bool dflt_shape = q.diamond_width == 0 && q.cells_per_lane == 0 && q.threads_x == 0;
        const int nf = q.wavefront_depth ? q.wavefront_depth : (dflt_shape ? dnf : 1);
        if (nf < 0) return GIRIH_E_INVALID;
        // (so is the default schedule: variant 0 with the default shape means "default")
        if (dflt_shape && q.variant == 0 && q.wavefront_depth == 0) q.variant = dvar;
        // variant bit 0: dependency-driven schedule; bit 1: relaxed
        // synchronisation within the tile
        if (q.variant < 0 || q.variant > 3) return GIRIH_E_INVALID;
        const KernelEntry* k = find_mwd(p->stencil, p->dtype, dw, vx, wx, nf, (q.variant >> 1) & 1);
        if (!k) return GIRIH_E_UNSUPPORTED;
        if ((q.variant & 1) && !k->launch_sweep) return GIRIH_E_UNSUPPORTED;
        // the kernel addresses a window of nf*(RZ*(L+1)+1) planes (RZ = ceil(R/nf))
        // with 32-bit offsets
        const int64_t rz = p->stencil == GIRIH_27PT_BOX ? 2 : (R + nf - 1) / nf;   // level skew in slabs
        const int64_t win = (int64_t)nf * (rz * (dw / R + 1) + 1);
        if (win * p->grid.pitch_y * p->grid.pitch_x * (int64_t)elem_bytes(p->dtype) >= (int64_t)1 << 31)
            return GIRIH_E_UNSUPPORTED;
        int64_t xo = q.tile_x ? q.tile_x : default_x_tile(p, k, dw);
        if (xo <= 0) return GIRIH_E_INVALID;
        if (xo > k->xown_max) return GIRIH_E_LDS;
        if (xo > p->grid.nx) xo = std::max<int64_t>(1, p->grid.nx);
        p->kern = k;
        p->x_own = xo;
        p->n_xchunks = (p->grid.nx + xo - 1) / xo;
        q.diamond_width = dw;
        q.wavefront_depth = nf;
        q.tile_x = (int32_t)xo;
        q.tile_y = dw;
        q.tile_z = (int32_t)std::min<int64_t>(p->grid.nz, INT32_MAX);
        q.threads_x = 64 * wx;
        q.cells_per_lane = vx;
        q.threads_y = dw / 2;
    } else {
        // Defaults (measured on the 512^3, 384^3 and 256x512x1024 workloads):
        // plane tiles in LDS of 64 x 16 cells marching up to 128 planes;
        // register columns for the box stencil (1.6x the cached variant in
        // FP64, 1.5x in FP32) and, in FP32, for the constant-coefficient star
        // stencils (7-point 1.3x the cached variant, 25-point 1.26x the plane
        // tiles; in FP64 they tie or lose).  The z chunk keeps at least two
        // blocks per CU on small grids.
        const bool dflt = !in || (in->threads_x == 0 && in->threads_y == 0 && in->variant == 0);
        const bool box = p->stencil == GIRIH_27PT_BOX;
        if (dflt) {
            const bool f32 = p->dtype == GIRIH_F32;
            const bool scols = f32 && (p->stencil == GIRIH_7PT_CONST || p->stencil == GIRIH_25PT_CONST);
            q.threads_x = 64;
            q.threads_y = 16;
            q.variant = 1;
            int64_t cap = 128;
            if (box) {
                // 2 waves per block of 8 rows (FP64) or 4 rows (FP32), z chunks
                // of up to 32 (FP64) or 12 (FP32) planes
                q.threads_y = 2;
                if (q.cells_per_lane == 0) q.cells_per_lane = f32 ? 4 : 8;
                cap = f32 ? 12 : 32;
            } else if (scols) {
                // 2 waves per block of 4 (7-point) or 8 (25-point) rows, z
                // chunks of up to 12 planes
                q.threads_y = 2;
                q.variant = 2;
                if (q.cells_per_lane == 0) q.cells_per_lane = p->stencil == GIRIH_7PT_CONST ? 4 : 8;
                cap = 12;
            }
            if (q.tile_z == 0) {
                // columns of blocks (register columns: of waves)
                const int64_t own = 64 - 2 * kRadius[p->stencil];
                const int64_t cols = box || scols
                                         ? ((p->grid.nx + own - 1) / own) * ((p->grid.ny + q.cells_per_lane - 1) / q.cells_per_lane)
                                         : ((p->grid.nx + 63) / 64) * ((p->grid.ny + q.threads_y - 1) / q.threads_y);
                const int64_t tz = cols * p->grid.nz / 512;
                q.tile_z = (int32_t)std::max<int64_t>(std::min<int64_t>(8, cap), std::min<int64_t>(cap, tz));
            }
        }
        if (q.threads_x == 0) q.threads_x = 64;
        if (q.threads_y == 0) q.threads_y = 4;
        if (q.tile_z == 0) q.tile_z = 64;
        if (q.threads_x <= 0 || q.threads_y <= 0 || q.tile_z <= 0) return GIRIH_E_INVALID;
        if (q.variant < 0 || q.variant > 2) return GIRIH_E_UNSUPPORTED;
        if (q.variant == 0 && (q.threads_x * q.threads_y > 256 || q.threads_x % 64)) return GIRIH_E_INVALID;
        if (q.variant >= 1 && q.threads_x != 64) return GIRIH_E_INVALID;
        // register columns: variant 1 of the box stencil, variant 2 of the
        // constant-coefficient star stencils
        const bool cols = (box && q.variant == 1) || q.variant == 2;
        if (cols && q.cells_per_lane == 0) q.cells_per_lane = 4;
        p->kern = find_naive(p->stencil, p->dtype, q.variant, q.threads_y, cols ? q.cells_per_lane : 0);
        if (!p->kern) return GIRIH_E_UNSUPPORTED;
        q.diamond_width = 0;
        q.wavefront_depth = 0;
        // x and y cells a block stores (register columns: 64 - 2R lanes of
        // each wave, cells_per_lane rows per lane)
        q.tile_x = cols ? 64 - 2 * kRadius[p->stencil] : q.threads_x;
        q.tile_y = cols ? q.threads_y * q.cells_per_lane : q.threads_y;
        if (!cols) q.cells_per_lane = 1;
    }
    p->params = q;
    return GIRIH_OK;
}

template <typename Real>
void fill_coefs(const girih_plan_s* p, const void* const* arrays, CoefArgs<Real>& c) {
    for (int m = 0; m < 13; ++m) c.arr[m] = nullptr;
    for (int m = 0; m < 5; ++m) c.k[m] = (Real)p->consts[m];
    for (int m = 0; m < kNCoef[p->stencil]; ++m) c.arr[m] = static_cast<const Real*>(arrays[m]);
}

GridDesc desc_of(const girih_plan_s* p) {
    GridDesc g;
    g.nx = p->grid.nx;
    g.ny = p->grid.ny;
    g.nz = p->grid.nz;
    g.pitch_x = p->grid.pitch_x;
    g.pitch_y = p->grid.pitch_y;
    g.h = p->grid.halo;
    return g;
}

#define HIPCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return GIRIH_E_HIP;  \
    } while (0)

// Launch one sweep kernel; with timing on, bracket it with a pair of events
// on the same stream.
int timed_launch(girih_plan_s* p, LaunchFn launch, const void* args, dim3 grid, dim3 block, hipStream_t s) {
    if (!p->timing) return launch(args, grid, block, s) == hipSuccess ? GIRIH_OK : GIRIH_E_HIP;
    const size_t need = 2 * (size_t)(p->n_timed + 1);
    while (p->events.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return GIRIH_E_HIP;
        p->events.push_back(e);
    }
    HIPCHK(hipEventRecord(p->events[2 * p->n_timed], s));
    HIPCHK(launch(args, grid, block, s));
    HIPCHK(hipEventRecord(p->events[2 * p->n_timed + 1], s));
    ++p->n_timed;
    return GIRIH_OK;
}

template <typename Real>
int run_naive(girih_plan_s* p, void* buf0, void* buf1, const void* const* coefs, int64_t T, hipStream_t s,
              bool timed) {
    NaiveArgs<Real> a;
    a.g = desc_of(p);
    fill_coefs<Real>(p, coefs, a.coef);
    a.z_chunk = p->params.tile_z;
    // XCD-contiguous tile runs: measured faster for 7c, 25c and 7v (+4..7 %),
    // within 2 % for the second-order 25-point stencil, and slower for the 15
    // domain-sized streams of 25v (-16 %)
    a.xcd_runs = kStreams[p->stencil] <= 9 ? 1 : 0;
    const dim3 block(p->params.threads_x, p->params.threads_y);
    const int64_t bx = p->params.tile_x, by = p->params.tile_y;   // cells a block stores along x and y
    const dim3 grid((unsigned)((p->grid.nx + bx - 1) / bx), (unsigned)((p->grid.ny + by - 1) / by),
                    (unsigned)((p->grid.nz + a.z_chunk - 1) / a.z_chunk));
    Real* b[2] = {static_cast<Real*>(buf0), static_cast<Real*>(buf1)};
    for (int64_t t = 0; t < T; ++t) {
        a.V = b[t & 1];
        a.U = b[(t + 1) & 1];
        const int rc = timed ? timed_launch(p, p->kern->launch, &a, grid, block, s)
                             : (p->kern->launch(&a, grid, block, s) == hipSuccess ? GIRIH_OK : GIRIH_E_HIP);
        if (rc) return rc;
    }
    return GIRIH_OK;
}

int ensure_work(girih_plan_s* p) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const size_t need = grid_bytes(p);
    if (p->work[0] && p->work_bytes == need && p->work_device == dev) return GIRIH_OK;
    for (int i = 0; i < 2; ++i) {
        if (p->work[i]) (void)hipFree(p->work[i]);
        p->work[i] = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        if (hipMalloc(&p->work[i], need) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < 2; ++j) {
                if (p->work[j]) (void)hipFree(p->work[j]);
                p->work[j] = nullptr;
            }
            return GIRIH_E_NOMEM;
        }
    }
    if (p->halo_flag) (void)hipFree(p->halo_flag);
    p->halo_flag = nullptr;
    if (hipMalloc(&p->halo_flag, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        return GIRIH_E_NOMEM;
    }
    p->work_bytes = need;
    p->work_device = dev;
    return GIRIH_OK;
}

// Device memory a run uses beside the caller's buffers: the MWD pair (two
// arrays of the grid's size) and the one-int halo flag.
struct RunWork {
    void* arr[2];
    int* flag;
    uint32_t* error;   // error word of bounded waits (null: allocate the plan's)
};

// Device state of the dependency-driven schedule: kSchedHead words (the
// queue counters, then the error word) and four rows of completion marks.
constexpr int kSchedHead = 16;
constexpr int kSchedError = 8;

__global__ void sched_reset_kernel(uint32_t* head) {
    if (threadIdx.x < kSchedHead) head[threadIdx.x] = 0;
}

__global__ void zero_u32_kernel(uint32_t* a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

int ensure_sched(girih_plan_s* p, int64_t tpr, hipStream_t s) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const int64_t need = kSchedHead + 4 * tpr;
    if (p->sched && p->sched_words >= need && p->sched_device == dev) return GIRIH_OK;
    if (p->sched) (void)hipFree(p->sched);
    p->sched = nullptr;
    if (hipMalloc(&p->sched, (size_t)need * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return GIRIH_E_NOMEM;
    }
    // marks start below every run's base
    hipLaunchKernelGGL(zero_u32_kernel, dim3(64), dim3(256), 0, s, p->sched, need);
    HIPCHK(hipGetLastError());
    p->sched_words = need;
    p->sched_device = dev;
    p->sched_base = 1;
    return GIRIH_OK;
}

template <typename Real>
int run_mwd(girih_plan_s* p, void* buf0, void* buf1, const void* const* coefs, int64_t T, hipStream_t s,
            const RunWork& w, bool timed) {
    int rc = GIRIH_OK;
    const int64_t nx = p->grid.nx, ny = p->grid.ny, nz = p->grid.nz, h = p->grid.halo;
    const int64_t px = p->grid.pitch_x, py = p->grid.pitch_y;
    const int eb = (int)sizeof(Real);
    // every array carries buf0's fixed halo
    HIPCHK(launch_copy_halo(buf0, w.arr[0], eb, nx, ny, nz, h, px, py, s));
    HIPCHK(launch_copy_halo(buf0, w.arr[1], eb, nx, ny, nz, h, px, py, s));
    HIPCHK(launch_zero_halo_flag(buf0, w.flag, eb, nx, ny, nz, h, px, py, s));
    const int dw = p->kern->dw;
    const int64_t H = dw / (2 * p->R);
    const int64_t n_rows = (T - 1) / H + 2;
    Real* user[2] = {static_cast<Real*>(buf0), static_cast<Real*>(buf1)};
    Real* scr[2] = {static_cast<Real*>(w.arr[0]), static_cast<Real*>(w.arr[1])};
    // The last row must write the caller's pair: rows alternate in -> out, so
    // row 0 reads the caller's pair iff the row count is even; otherwise u^0
    // is first copied into the other pair.
    bool in_user = (n_rows % 2) == 0;
    if (!in_user) {
        HIPCHK(hipMemcpyAsync(scr[0], user[0], grid_bytes(p), hipMemcpyDeviceToDevice, s));
        // second-order-in-time stencils: the second buffer holds u^{-1}
        if (p->stencil == GIRIH_25PT_LEAPFROG)
            HIPCHK(hipMemcpyAsync(scr[1], user[1], grid_bytes(p), hipMemcpyDeviceToDevice, s));
    }
    MwdArgs<Real> a;
    a.g = desc_of(p);
    fill_coefs<Real>(p, coefs, a.coef);
    a.T = T;
    a.x_own = (int32_t)p->x_own;
    a.zero_halo = w.flag;
    a.spin_limit = p->spin_limit;
    a.error = nullptr;
    p->err_word = nullptr;
    const bool sweep = (p->params.variant & 1) && timed;
    if (p->kern->sync || sweep) {
        // bounded waits report to an error word, cleared by a kernel
        // (capturable) before the run
        if (w.error) {
            a.error = w.error;
        } else {
            rc = ensure_sched(p, 1, s);
            if (rc) return rc;
            a.error = p->sched + kSchedError;
        }
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, a.error, (int64_t)1);
        HIPCHK(hipGetLastError());
        p->err_word = a.error;
    }
    const dim3 block(p->kern->nthreads);
    if (sweep) {
        // one dependency-driven launch for every row (the fixed-scratch
        // entry point keeps the row launches: it has no room for the marks)
        MwdSweepArgs<Real> sa;
        Real** even_in = in_user ? user : scr;   // row 0 reads this pair
        Real** odd_in = in_user ? scr : user;
        for (int par = 0; par < 2; ++par) {
            MwdArgs<Real>& ra = sa.rows[par];
            ra = a;
            Real** in = par ? odd_in : even_in;
            Real** out = par ? even_in : odd_in;
            ra.in[0] = in[0];
            ra.in[1] = in[1];
            ra.out[0] = out[0];
            ra.out[1] = out[1];
            ra.t_c = 0;   // per row, from the row index
            ra.c_first = par ? dw / 2 : 0;
        }
        SweepSched& sc = sa.s;
        const int R = p->R, L = dw / R;
        sc.n_chunks = (int32_t)p->n_xchunks;
        sc.nd[0] = (int32_t)((ny + dw / 2 + dw - 1) / dw);
        sc.nd[1] = (int32_t)((ny + dw - 1) / dw);
        for (int par = 0; par < 2; ++par) sc.nb[par] = (sc.nd[par] * sc.n_chunks + 7) / 8 * 8;
        sc.tpr = std::max(sc.nd[0], sc.nd[1]) * sc.n_chunks;
        sc.H = (int32_t)H;
        // x chunks whose cells a tile reads, or whose reads its stores
        // overwrite: within ceil((XL - HX + R) / x_own) - 1 of its own
        const int64_t XL = 64 * (int64_t)p->kern->vx * p->kern->wx, HX = (int64_t)R * (L - 1);
        sc.kx = (int32_t)std::max<int64_t>(1, (XL - HX + R + p->x_own - 1) / p->x_own - 1);
        // rows that fit the clipped-slot body (where the shape has one)
        sc.clip_lo = 0;
        sc.clip_hi = (int32_t)n_rows;
        if (H + 3 < 2 * H + 2) {
            int64_t lo = n_rows, hi = -1;
            for (int64_t r = 0; r < n_rows; ++r)
                if (mwd_slots_needed(R, dw, r * H, T) > H + 3) {
                    lo = std::min(lo, r);
                    hi = r;
                }
            sc.clip_lo = (int32_t)lo;
            sc.clip_hi = (int32_t)(hi < 0 ? n_rows : hi + 1);
        }
        rc = ensure_sched(p, sc.tpr, s);
        if (rc) return rc;
        sc.error = p->sched + kSchedError;
        for (int par = 0; par < 2; ++par) sa.rows[par].error = sc.error;
        p->err_word = sc.error;
        sc.done = p->sched + kSchedHead;
        sc.base = p->sched_base;
        p->sched_base += (uint32_t)n_rows + 4;
        sc.spin_limit = p->spin_limit;
        hipLaunchKernelGGL(sched_reset_kernel, dim3(1), dim3(64), 0, s, p->sched);
        HIPCHK(hipGetLastError());
        const int64_t blocks = (n_rows / 2) * (sc.nb[0] + sc.nb[1]) + (n_rows & 1 ? sc.nb[0] : 0);
        return timed_launch(p, p->kern->launch_sweep, &sa, dim3((unsigned)blocks), block, s);
    }
    for (int64_t r = 0; r < n_rows; ++r) {
        Real** in = in_user ? user : scr;
        Real** out = in_user ? scr : user;
        a.in[0] = in[0];
        a.in[1] = in[1];
        a.out[0] = out[0];
        a.out[1] = out[1];
        a.t_c = r * H;
        const int64_t off = (r & 1) ? dw / 2 : 0;
        a.c_first = off;
        const int64_t n_diamonds = (ny + dw / 2 - off + dw - 1) / dw;
        const dim3 grid((unsigned)p->n_xchunks, (unsigned)n_diamonds);
        const KernelEntry* k = mwd_kernel_for(p->kern, mwd_slots_needed(p->R, dw, a.t_c, T));
        rc = timed ? timed_launch(p, k->launch, &a, grid, block, s)
                   : (k->launch(&a, grid, block, s) == hipSuccess ? GIRIH_OK : GIRIH_E_HIP);
        if (rc) return rc;
        in_user = !in_user;
    }
    return GIRIH_OK;
}

int validate_grid(const girih_grid* g, int R, girih_grid& out) {
    if (!g) return GIRIH_E_INVALID;
    out = *g;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->halo != R) return GIRIH_E_INVALID;
    if (out.pitch_x == 0) out.pitch_x = g->nx + 2 * R;
    if (out.pitch_y == 0) out.pitch_y = g->ny + 2 * R;
    if (out.pitch_x < g->nx + 2 * R || out.pitch_y < g->ny + 2 * R) return GIRIH_E_INVALID;
    // kernel grid dimensions: y of the haloed box and diamonds per row fit 16 bits of gridDim
    if (g->ny + 2 * R > 65535 || g->nz + 2 * R > 65535) return GIRIH_E_UNSUPPORTED;
    return GIRIH_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ tuner

struct TuneBufs {
    void* f[2] = {nullptr, nullptr};
    std::vector<void*> coef;
    ~TuneBufs() {
        for (void* q : f)
            if (q) (void)hipFree(q);
        for (void* q : coef)
            if (q) (void)hipFree(q);
    }
};

template <typename Real>
__global__ void tune_fill_kernel(Real* __restrict__ a, int64_t n, Real v, uint32_t seed, int64_t px, int64_t py,
                                 int64_t nx, int64_t ny, int64_t nz, int h, int zero_halo) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (zero_halo) {
            // the tuner's fields carry a zero Dirichlet halo, like the workloads
            const int64_t x = i % px, y = (i / px) % py, z = i / (px * py);
            if (x < h || x >= nx + h || y < h || y >= ny + h || z < h || z >= nz + h) {
                a[i] = Real(0);
                continue;
            }
        }
        // cheap hash in [0.5, 1.5) * v : keeps values normal and bounded
        uint32_t x = (uint32_t)i * 2654435761u ^ seed;
        x ^= x >> 15;
        x *= 2246822519u;
        x ^= x >> 13;
        a[i] = v * (Real)(0.5 + (double)(x & 0xffffff) / 16777216.0);
    }
}

int alloc_tune_bufs(girih_plan_s* p, TuneBufs& b, hipStream_t s) {
    const size_t bytes = grid_bytes(p);
    const int64_t n = (int64_t)(bytes / elem_bytes(p->dtype));
    const int nc = kNCoef[p->stencil];
    b.coef.assign(nc, nullptr);
    for (int i = 0; i < 2; ++i)
        if (hipMalloc(&b.f[i], bytes) != hipSuccess) { (void)hipGetLastError(); return GIRIH_E_NOMEM; }
    for (int i = 0; i < nc; ++i)
        if (hipMalloc(&b.coef[i], bytes) != hipSuccess) { (void)hipGetLastError(); return GIRIH_E_NOMEM; }
    const double cw = nc ? 1.0 / (nc == 7 ? 7.0 : 25.0) : 0.0;
    for (int i = 0; i < 2 + nc; ++i) {
        void* q = i < 2 ? b.f[i] : b.coef[i - 2];
        const double v = i < 2 ? 1.0 : cw;
        if (p->dtype == GIRIH_F64)
            hipLaunchKernelGGL(tune_fill_kernel<double>, dim3(4096), dim3(256), 0, s, (double*)q, n, v, 17u * i + 1,
                               p->grid.pitch_x, p->grid.pitch_y, p->grid.nx, p->grid.ny, p->grid.nz, p->grid.halo,
                               i < 2 ? 1 : 0);
        else
            hipLaunchKernelGGL(tune_fill_kernel<float>, dim3(4096), dim3(256), 0, s, (float*)q, n, (float)v, 17u * i + 1,
                               p->grid.pitch_x, p->grid.pitch_y, p->grid.nx, p->grid.ny, p->grid.nz, p->grid.halo,
                               i < 2 ? 1 : 0);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    return GIRIH_OK;
}

int run_any(girih_plan_s* p, void* b0, void* b1, const void* const* coefs, int64_t T, hipStream_t s,
            const RunWork* fixed = nullptr);

// Adaptive test length (paper, Section "Auto-tuning": test runs are
// lengthened until the measurement is stable).  time_reps(k) returns the
// seconds of k back-to-back runs of the problem (negative: failure).  The
// repeat count k doubles while a measurement is shorter than min_seconds;
// the per-run time is accepted when two consecutive measurements agree
// within tol (relative), or when max_seconds or max_tries is reached (the
// last measurement is then taken).
struct Adapted {
    double per_run = 0;   // seconds per run of the accepted measurement
    int64_t reps = 0;     // runs in it
    int tries = 0;        // measurements taken
    int status = GIRIH_OK;
};

template <class F>
Adapted adaptive_time(F&& time_reps, double tol, double min_seconds, double max_seconds, int max_tries) {
    Adapted r;
    int64_t reps = 1;
    double prev = -1;
    const double t0 = now_s();
    for (;;) {
        const double secs = time_reps(reps);
        if (!(secs >= 0)) {
            r.status = GIRIH_E_HIP;
            return r;
        }
        ++r.tries;
        const double per = secs / (double)reps;
        r.per_run = per;
        r.reps = reps;
        if (prev > 0 && std::fabs(per - prev) <= tol * std::max(per, prev)) break;
        if (now_s() - t0 > max_seconds || r.tries >= max_tries) break;
        prev = per;
        if (secs < min_seconds) reps *= 2;
    }
    return r;
}

// Time one candidate on the problem it is tuned for: back-to-back runs of the
// plan's own T-step schedule (every diamond row, the clipped first and last
// rows included), with the adaptive length above (3 %, runs of at least
// 50 ms).
int measure(girih_plan_s* p, TuneBufs& b, hipStream_t s, int64_t T, double max_seconds, girih_tune_record& rec) {
    const double lups = (double)p->grid.nx * p->grid.ny * p->grid.nz * (double)T;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return GIRIH_E_HIP;
    }
    const void* const* coefs = b.coef.empty() ? nullptr : (const void* const*)b.coef.data();
    // warm-up (also allocates the plan's pair)
    int rc = run_any(p, b.f[0], b.f[1], coefs, T, s);
    if (rc == GIRIH_OK && hipStreamSynchronize(s) != hipSuccess) rc = GIRIH_E_HIP;
    Adapted ad;
    if (rc == GIRIH_OK) {
        ad = adaptive_time(
            [&](int64_t reps) -> double {
                if (hipEventRecord(e0, s) != hipSuccess) return -1;
                for (int64_t i = 0; i < reps; ++i) {
                    rc = run_any(p, b.f[0], b.f[1], coefs, T, s);
                    if (rc) return -1;
                }
                float ms = 0;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    return -1;
                return ms * 1e-3;
            },
            0.03, 0.05, max_seconds, 12);
        if (rc == GIRIH_OK) rc = ad.status;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rec.params = p->params;
    rec.lds_bytes = p->kern->lds_bytes;
    rec.steps = T * ad.reps;
    rec.seconds = ad.per_run * (double)ad.reps;
    rec.glups = rc == GIRIH_OK && ad.per_run > 0 ? lups / ad.per_run * 1e-9 : 0;
    rec.repeats = ad.tries;
    rec.status = rc;
    return rc;
}

// The tuner's search over a candidate list, with any measurement
// (measure(i) -> GLUP/s of candidate i, <= 0 when it fails).
//  exhaustive (and model): every candidate in list order until max_seconds
//  is spent (at least one);
//  hill climbing (paper, Section "Auto-tuning"): per thread shape (waves
//  along x and cells per lane), start at the median diamond width and the
//  widest x tile of the smallest wavefront depth and move to the best
//  improving neighbour until none improves: the next diamond width or
//  wavefront depth up or down (at the widest x tile there), or the next x
//  tile up or down at the same width and depth.
// Returns the index of the best candidate (-1 if none measured).
template <class M>
int tune_search(const std::vector<girih_params>& cands, int mode, M&& measure_i, double max_seconds,
                double& best_rate, int& n_measured) {
    const double t_start = now_s();
    std::vector<double> rate(cands.size(), -1.0);
    best_rate = -1;
    n_measured = 0;
    int best_i = -1;
    auto eval = [&](int i) -> double {
        if (rate[i] < 0) {
            const double r = measure_i(i);
            rate[i] = r > 0 ? r : 0;
            ++n_measured;
            if (rate[i] > best_rate) {
                best_rate = rate[i];
                best_i = i;
            }
        }
        return rate[i];
    };
    if (mode != GIRIH_TUNE_HILLCLIMB) {
        for (size_t i = 0; i < cands.size(); ++i) {
            if (n_measured > 0 && now_s() - t_start > max_seconds) break;
            eval((int)i);
        }
        return best_rate > 0 ? best_i : -1;
    }
    std::map<std::pair<int, int>, std::vector<int>> by_shape;
    for (size_t i = 0; i < cands.size(); ++i)
        by_shape[{cands[i].threads_x * 4 + cands[i].variant, cands[i].cells_per_lane}].push_back((int)i);
    for (auto& kv : by_shape) {
        const std::vector<int>& g = kv.second;
        std::vector<int> dws, nfs;
        for (int i : g) {
            dws.push_back(cands[i].diamond_width);
            nfs.push_back(std::max(1, cands[i].wavefront_depth));
        }
        std::sort(dws.begin(), dws.end());
        dws.erase(std::unique(dws.begin(), dws.end()), dws.end());
        std::sort(nfs.begin(), nfs.end());
        nfs.erase(std::unique(nfs.begin(), nfs.end()), nfs.end());
        auto nf_of = [&](int i) { return std::max(1, cands[i].wavefront_depth); };
        // candidates of one (diamond width, depth), by x tile
        auto tiles = [&](int dw, int nf) {
            std::vector<int> t;
            for (int i : g)
                if (cands[i].diamond_width == dw && nf_of(i) == nf) t.push_back(i);
            std::sort(t.begin(), t.end(), [&](int a, int b) { return cands[a].tile_x < cands[b].tile_x; });
            return t;
        };
        // start: median width (with a candidate at the smallest depth), widest tile
        int cur = -1;
        for (size_t d = dws.size() / 2, n = 0; n < dws.size() && cur < 0; ++n) {
            const size_t di = (d + n) % dws.size();
            for (int nf : nfs) {
                auto t = tiles(dws[di], nf);
                if (!t.empty()) { cur = t.back(); break; }
            }
        }
        if (cur < 0) continue;
        double cv = eval(cur);
        for (int guard = 0; guard < 256; ++guard) {
            if (now_s() - t_start > max_seconds) break;
            const int dw = cands[cur].diamond_width, nf = nf_of(cur);
            const int di = (int)(std::find(dws.begin(), dws.end(), dw) - dws.begin());
            const int fi = (int)(std::find(nfs.begin(), nfs.end(), nf) - nfs.begin());
            std::vector<int> nb;
            for (int d : {-1, 1}) {
                if (di + d >= 0 && di + d < (int)dws.size()) {
                    auto t = tiles(dws[di + d], nf);
                    if (!t.empty()) nb.push_back(t.back());
                }
                if (fi + d >= 0 && fi + d < (int)nfs.size()) {
                    auto t = tiles(dw, nfs[fi + d]);
                    if (!t.empty()) nb.push_back(t.back());
                }
            }
            auto t = tiles(dw, nf);
            const int ti = (int)(std::find(t.begin(), t.end(), cur) - t.begin());
            if (ti > 0) nb.push_back(t[ti - 1]);
            if (ti + 1 < (int)t.size()) nb.push_back(t[ti + 1]);
            int bi = cur;
            double bv = cv;
            for (int i : nb) {
                const double r = eval(i);
                if (r > bv) { bv = r; bi = i; }
            }
            if (bi == cur) break;
            cur = bi;
            cv = bv;
        }
    }
    return best_rate > 0 ? best_i : -1;
}

std::vector<girih_params> mwd_candidates(const girih_plan_s* p) {
    std::vector<girih_params> out;
    for (const auto& e : kernel_table()) {
        if (e.algo != AL_MWD || e.stencil != p->stencil || e.dtype != p->dtype || e.ns != 0) continue;
        if (e.xown_max < 8) continue;
        if (p->lds_budget > 0 && e.lds_bytes > p->lds_budget) continue;
        // x tiles: the widest, and the widths that split nx into 1-3 more chunks
        std::set<int64_t> tiles;
        const int64_t nx = p->grid.nx;
        const int64_t c0 = (nx + e.xown_max - 1) / e.xown_max;
        for (int64_t c = c0; c <= c0 + 3; ++c) {
            const int64_t t = (nx + c - 1) / c;
            if (t >= 8 && t <= e.xown_max) tiles.insert(t);
        }
        for (int64_t t : tiles) {
            girih_params q{};
            q.diamond_width = e.dw;
            q.wavefront_depth = e.nf;
            q.tile_x = (int32_t)t;
            q.threads_x = 64 * e.wx;
            q.cells_per_lane = e.vx;
            q.threads_y = e.dw / 2;
            q.variant = e.sync ? 2 : 0;
            out.push_back(q);
            if (e.launch_sweep) {
                q.variant |= 1;
                out.push_back(q);
            }
        }
    }
    return out;
}

std::vector<girih_params> naive_candidates(const girih_plan_s*) {
    std::vector<girih_params> out;
    const int tx[] = {64, 128, 256};
    const int ty[] = {1, 2, 4};
    const int tz[] = {16, 64, 256};
    for (int a : tx)
        for (int b : ty)
            for (int c : tz) {
                if (a * b > 256) continue;
                girih_params q{};
                q.threads_x = a;
                q.threads_y = b;
                q.tile_z = c;
                out.push_back(q);
            }
    // plane tiles in LDS: 64 x rows threads
    const int rows[] = {4, 8, 16};
    const int tz1[] = {64, 128, 256};
    for (int b : rows)
        for (int c : tz1) {
            girih_params q{};
            q.threads_x = 64;
            q.threads_y = b;
            q.tile_z = c;
            q.variant = 1;
            out.push_back(q);
        }
    return out;
}

}  // namespace

namespace {
int run_any(girih_plan_s* p, void* b0, void* b1, const void* const* coefs, int64_t T, hipStream_t s,
            const RunWork* fixed) {
    p->err_word = nullptr;
    if (T == 0) return GIRIH_OK;
    RunWork w{{nullptr, nullptr}, nullptr, nullptr};
    if (p->algo == GIRIH_MWD) {
        if (fixed) {
            w = *fixed;
        } else {
            const int rc = ensure_work(p);
            if (rc) return rc;
            w = RunWork{{p->work[0], p->work[1]}, p->halo_flag, nullptr};
        }
    }
    const bool timed = fixed == nullptr;
    HIPCHK(launch_copy_halo(b0, b1, (int)elem_bytes(p->dtype), p->grid.nx, p->grid.ny, p->grid.nz, p->grid.halo,
                            p->grid.pitch_x, p->grid.pitch_y, s));
    if (p->algo == GIRIH_NAIVE)
        return p->dtype == GIRIH_F64 ? run_naive<double>(p, b0, b1, coefs, T, s, timed)
                                     : run_naive<float>(p, b0, b1, coefs, T, s, timed);
    return p->dtype == GIRIH_F64 ? run_mwd<double>(p, b0, b1, coefs, T, s, w, timed)
                                 : run_mwd<float>(p, b0, b1, coefs, T, s, w, timed);
}
}  // namespace

// ------------------------------------------------ fixed scratch (no allocation)

// Device memory of girih_run_noalloc, for callers that cannot allocate: the
// halo flag (first 256 bytes), then the MWD pair of at most kFixedArrayBytes
// each.  Every device the library runs on holds one copy for the life of the
// process; all calls on one device share it.
constexpr size_t kFixedFlagBytes = 256;
constexpr size_t kFixedErrorOffset = 128;   // error word of bounded waits, within the flag bytes
constexpr size_t kFixedArrayBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kFixedFlagBytes + 2 * kFixedArrayBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (the array's name is only a host-side handle).
int fixed_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return GIRIH_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return GIRIH_E_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GIRIH_OK;
}
}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int girih_plan(girih_plan_t* out, girih_stencil stencil, girih_dtype dtype, const girih_grid* grid,
               const double* const_coefs, girih_algo algo, const girih_params* params) {
    if (!out) return GIRIH_E_INVALID;
    *out = nullptr;
    if ((int)stencil < 0 || (int)stencil >= kNStencils || (dtype != GIRIH_F64 && dtype != GIRIH_F32) ||
        (algo != GIRIH_NAIVE && algo != GIRIH_MWD))
        return GIRIH_E_INVALID;
    girih_grid g;
    int rc = validate_grid(grid, kRadius[stencil], g);
    if (rc) return rc;
    if (kNConst[stencil] && !const_coefs) return GIRIH_E_INVALID;
    girih_plan_s* p = new (std::nothrow) girih_plan_s();
    if (!p) return GIRIH_E_NOMEM;
    p->stencil = stencil;
    p->dtype = dtype;
    p->algo = algo;
    p->grid = g;
    p->R = kRadius[stencil];
    for (int m = 0; m < kNConst[stencil]; ++m) {
        const double c = const_coefs[m];
        if (!std::isfinite(c)) { delete p; return GIRIH_E_INVALID; }
        p->consts[m] = dtype == GIRIH_F32 ? (double)(float)c : c;
    }
    rc = resolve(p, params);
    if (rc) { delete p; return rc; }
    *out = p;
    return GIRIH_OK;
}

int girih_plan_set_params(girih_plan_t p, const girih_params* params) {
    if (!p) return GIRIH_E_INVALID;
    girih_plan_s tmp = *p;
    tmp.work[0] = tmp.work[1] = nullptr;   // not owned by the copy
    tmp.sched = nullptr;
    tmp.halo_flag = nullptr;
    int rc = resolve(&tmp, params);
    if (rc) return rc;
    p->params = tmp.params;
    p->kern = tmp.kern;
    p->x_own = tmp.x_own;
    p->n_xchunks = tmp.n_xchunks;
    return GIRIH_OK;
}

int girih_run(girih_plan_t p, void* buf0, void* buf1, const void* const* coef_arrays, int32_t n_coef, int64_t T,
              void* hip_stream, int32_t* result_index) {
    if (!p || !buf0 || !buf1 || buf0 == buf1 || T < 0) return GIRIH_E_INVALID;
    if (n_coef != kNCoef[p->stencil]) return GIRIH_E_INVALID;
    if (n_coef && !coef_arrays) return GIRIH_E_INVALID;
    for (int m = 0; m < n_coef; ++m)
        if (!coef_arrays[m]) return GIRIH_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    p->n_timed = 0;   // the timing record covers the last run
    int rc = run_any(p, buf0, buf1, coef_arrays, T, s);
    if (rc) return rc;
    if (result_index) *result_index = (int32_t)(T & 1);
    return GIRIH_OK;
}

int girih_run_noalloc(girih_plan_t p, void* buf0, void* buf1, const void* const* coef_arrays, int32_t n_coef,
                      int64_t T, void* hip_stream, int32_t* result_index) {
    if (!p || !buf0 || !buf1 || buf0 == buf1 || T < 0) return GIRIH_E_INVALID;
    if (n_coef != kNCoef[p->stencil]) return GIRIH_E_INVALID;
    if (n_coef && !coef_arrays) return GIRIH_E_INVALID;
    for (int m = 0; m < n_coef; ++m)
        if (!coef_arrays[m]) return GIRIH_E_INVALID;
    if (p->algo == GIRIH_MWD && grid_bytes(p) > kFixedArrayBytes) return GIRIH_E_SCRATCH;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    RunWork w{{nullptr, nullptr}, nullptr, nullptr};
    if (p->algo == GIRIH_MWD && T > 0) {
        void* base = nullptr;
        const int rc = fixed_scratch(&base);
        if (rc) return rc;
        unsigned char* b = static_cast<unsigned char*>(base);
        w = RunWork{{b + kFixedFlagBytes, b + kFixedFlagBytes + kFixedArrayBytes}, reinterpret_cast<int*>(b),
                    reinterpret_cast<uint32_t*>(b + kFixedErrorOffset)};
    }
    p->n_timed = 0;
    const int rc = run_any(p, buf0, buf1, coef_arrays, T, s, &w);
    if (rc) return rc;
    if (result_index) *result_index = (int32_t)(T & 1);
    return GIRIH_OK;
}

int girih_tune_set_candidates(girih_plan_t p, const girih_params* cands, int32_t n) {
    if (!p || n < 0 || n > 4096 || (n && !cands)) return GIRIH_E_INVALID;
    p->tuning.model_cands.assign(cands, cands + n);
    return GIRIH_OK;
}

int girih_candidates(girih_plan_t p, girih_params* out, int32_t cap, int32_t* n) {
    if (!p || !n || cap < 0) return GIRIH_E_INVALID;
    auto c = p->algo == GIRIH_MWD ? mwd_candidates(p) : naive_candidates(p);
    *n = (int32_t)c.size();
    if (out)
        for (int32_t i = 0; i < cap && i < (int32_t)c.size(); ++i) out[i] = c[i];
    return GIRIH_OK;
}

int girih_tune(girih_plan_t p, int32_t mode, int64_t T, double max_seconds, void* hip_stream, girih_params* best,
               double* best_glups) {
    if (!p || T < 1 || !(max_seconds > 0)) return GIRIH_E_INVALID;
    if (mode < 0 || mode > 2) return GIRIH_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<girih_params> cands;
    if (mode == GIRIH_TUNE_MODEL) cands = p->tuning.model_cands;
    else cands = p->algo == GIRIH_MWD ? mwd_candidates(p) : naive_candidates(p);
    if (cands.empty()) return GIRIH_E_UNSUPPORTED;
    const girih_params saved = p->params;
    // the tuner's test runs are not recorded by the launch timing
    struct TimingOff {
        girih_plan_s* p;
        bool was;
        ~TimingOff() { p->timing = was; p->n_timed = 0; }
    } timing_off{p, p->timing};
    p->timing = false;
    TuneBufs bufs;
    int rc = alloc_tune_bufs(p, bufs, s);
    if (rc) return rc;
    const double per_cand = std::max(0.05, std::min(2.0, max_seconds / std::max<size_t>(cands.size(), 1)));
    std::vector<girih_params> resolved(cands.size());
    double best_rate = -1;
    int n_measured = 0;
    const int bi = tune_search(
        cands, p->algo == GIRIH_MWD ? mode : GIRIH_TUNE_EXHAUSTIVE,
        [&](int i) -> double {
            girih_tune_record rec{};
            rec.params = cands[i];
            int r2 = girih_plan_set_params(p, &cands[i]);
            if (r2 == GIRIH_OK) r2 = measure(p, bufs, s, T, per_cand, rec);
            rec.status = r2;
            if (r2 != GIRIH_OK) {
                (void)hipGetLastError();
                rec.glups = 0;
            }
            resolved[i] = p->params;
            p->tuning.log.push_back(rec);
            return rec.glups;
        },
        max_seconds, best_rate, n_measured);
    if (bi < 0) {
        (void)girih_plan_set_params(p, &saved);
        return GIRIH_E_UNSUPPORTED;
    }
    rc = girih_plan_set_params(p, &resolved[bi]);
    if (rc) return rc;
    if (best) *best = p->params;
    if (best_glups) *best_glups = best_rate;
    return GIRIH_OK;
}

int girih_tune_search(const girih_params* cands, int32_t n, int32_t mode, girih_measure_fn measure_fn, void* ctx,
                      double max_seconds, int32_t* best_index, double* best_glups, int32_t* n_measured) {
    if (!cands || n < 1 || !measure_fn || !(max_seconds > 0) || mode < 0 || mode > 2) return GIRIH_E_INVALID;
    std::vector<girih_params> c(cands, cands + n);
    double best = -1;
    int nm = 0;
    const int bi = tune_search(c, mode, [&](int i) { return measure_fn(&c[i], ctx); }, max_seconds, best, nm);
    if (best_index) *best_index = bi;
    if (best_glups) *best_glups = best;
    if (n_measured) *n_measured = nm;
    return bi < 0 ? GIRIH_E_UNSUPPORTED : GIRIH_OK;
}

int girih_adaptive_time(girih_time_fn time_fn, void* ctx, double tol, double min_seconds, double max_seconds,
                        int32_t max_tries, double* seconds_per_run, int64_t* reps, int32_t* tries) {
    if (!time_fn || !(tol >= 0) || !(max_seconds > 0) || max_tries < 1) return GIRIH_E_INVALID;
    const Adapted a = adaptive_time([&](int64_t k) { return time_fn(k, ctx); }, tol, min_seconds, max_seconds,
                                    max_tries);
    if (seconds_per_run) *seconds_per_run = a.per_run;
    if (reps) *reps = a.reps;
    if (tries) *tries = a.tries;
    return a.status;
}

int girih_tune_log(girih_plan_t p, girih_tune_record* out, int32_t cap, int32_t* n) {
    if (!p || !n || cap < 0) return GIRIH_E_INVALID;
    *n = (int32_t)p->tuning.log.size();
    if (out)
        for (int32_t i = 0; i < cap && i < *n; ++i) out[i] = p->tuning.log[i];
    return GIRIH_OK;
}

int girih_plan_info(girih_plan_t p, girih_params* params, int64_t* lds_bytes, double* model_bytes_per_lup) {
    if (!p) return GIRIH_E_INVALID;
    if (params) *params = p->params;
    if (lds_bytes) *lds_bytes = p->kern ? p->kern->lds_bytes : 0;
    if (model_bytes_per_lup) {
        const double s = (double)elem_bytes(p->dtype);
        if (p->algo == GIRIH_NAIVE) {
            *model_bytes_per_lup = kStreams[p->stencil] * s;
        } else {
            // paper's B_C in words: R*[(2Dw-2R) + (N_D*Dw+2R)] * 2 / Dw^2,
            // N_D = the pair of time levels + the coefficient arrays
            const int ND = 2 + kNCoef[p->stencil];
            const double Dw = p->params.diamond_width, R = p->R;
            *model_bytes_per_lup = 2 * s * R * ((2 * Dw - 2 * R) + (ND * Dw + 2 * R)) / (Dw * Dw);
        }
    }
    return GIRIH_OK;
}

int girih_set_lds_budget(girih_plan_t p, int64_t bytes) {
    if (!p || bytes < 0) return GIRIH_E_INVALID;
    p->lds_budget = bytes;
    return GIRIH_OK;
}

int girih_set_wait_limit(girih_plan_t p, uint32_t polls) {
    if (!p) return GIRIH_E_INVALID;
    p->spin_limit = polls;
    return GIRIH_OK;
}

int girih_check(girih_plan_t p, void* hip_stream) {
    if (!p) return GIRIH_E_INVALID;
    if (hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) != hipSuccess) return GIRIH_E_HIP;
    if (!p->err_word) return GIRIH_OK;
    uint32_t err = 0;
    if (hipMemcpy(&err, p->err_word, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return GIRIH_E_HIP;
    return err ? GIRIH_E_STALL : GIRIH_OK;
}

int girih_set_timing(girih_plan_t p, int32_t enable) {
    if (!p) return GIRIH_E_INVALID;
    p->timing = enable != 0;
    p->n_timed = 0;
    return GIRIH_OK;
}

int girih_timing(girih_plan_t p, int32_t* n_launches, double* kernel_ms) {
    if (!p || !n_launches || !kernel_ms) return GIRIH_E_INVALID;
    *n_launches = 0;
    *kernel_ms = 0;
    if (!p->timing || p->n_timed == 0) return GIRIH_OK;
    if (hipEventSynchronize(p->events[2 * p->n_timed - 1]) != hipSuccess) return GIRIH_E_HIP;
    double total = 0;
    for (int i = 0; i < p->n_timed; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p->events[2 * i], p->events[2 * i + 1]) != hipSuccess) return GIRIH_E_HIP;
        total += ms;
    }
    *n_launches = p->n_timed;
    *kernel_ms = total;
    return GIRIH_OK;
}

void girih_destroy(girih_plan_t p) {
    if (!p) return;
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i)
        if (p->work[i]) (void)hipFree(p->work[i]);
    if (p->halo_flag) (void)hipFree(p->halo_flag);
    if (p->sched) (void)hipFree(p->sched);
    delete p;
}

const char* girih_strerror(int code) {
    switch (code) {
        case GIRIH_OK: return "ok";
        case GIRIH_E_INVALID: return "invalid argument";
        case GIRIH_E_UNSUPPORTED: return "unsupported combination (no compiled kernel)";
        case GIRIH_E_LDS: return "tile exceeds the on-chip budget of the kernel";
        case GIRIH_E_HIP: return "HIP runtime error";
        case GIRIH_E_NOMEM: return "allocation failed";
        case GIRIH_E_NOGPU: return "no usable GPU";
        case GIRIH_E_SCRATCH: return "grid exceeds the fixed scratch of girih_run_noalloc (64 MiB per array)";
        case GIRIH_E_STALL: return "a dependency wait of the dependency-driven schedule gave up";
        default: return "unknown error";
    }
}

int girih_error_norms(const girih_grid* grid, girih_dtype dta, const void* a, girih_dtype dtb, const void* b,
                      void* hip_stream, double out[4]) {
    if (!grid || !a || !b || !out) return GIRIH_E_INVALID;
    if ((dta != GIRIH_F64 && dta != GIRIH_F32) || (dtb != GIRIH_F64 && dtb != GIRIH_F32)) return GIRIH_E_INVALID;
    const int64_t h = grid->halo;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || h < 0) return GIRIH_E_INVALID;
    const int64_t px = grid->pitch_x ? grid->pitch_x : grid->nx + 2 * h;
    const int64_t py = grid->pitch_y ? grid->pitch_y : grid->ny + 2 * h;
    if (px < grid->nx + 2 * h || py < grid->ny + 2 * h) return GIRIH_E_INVALID;
    if (error_norms(a, dta, b, dtb, grid->nx, grid->ny, grid->nz, h, px, py, static_cast<hipStream_t>(hip_stream),
                    out) != hipSuccess)
        return GIRIH_E_HIP;
    return GIRIH_OK;
}

const char* girih_version(void) { return "girih-mi355x 0.1 (gfx950)"; }

}  // extern "C"
