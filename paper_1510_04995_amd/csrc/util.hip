// Utility kernels: halo copy between buffers, and double-precision error
// norms of a result against a reference (accumulated in double whatever the
// element types are).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "registry.hpp"

namespace girih {

// One block per (j, k) row of the haloed box; rows outside the interior are
// copied whole, interior rows only their 2h x-halo cells.
template <typename T>
__global__ void __launch_bounds__(64)
copy_halo_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t nx, int64_t ny, int64_t nz,
                 int64_t h, int64_t pitch_x, int64_t pitch_y) {
    const int64_t jj = blockIdx.x;   // 0 .. ny+2h-1
    const int64_t kk = blockIdx.y;   // 0 .. nz+2h-1
    const int64_t base = (kk * pitch_y + jj) * pitch_x;
    const bool whole = kk < h || kk >= nz + h || jj < h || jj >= ny + h;
    if (whole) {
        for (int64_t i = threadIdx.x; i < nx + 2 * h; i += blockDim.x) dst[base + i] = src[base + i];
    } else if (threadIdx.x < 2 * h) {
        const int64_t i = threadIdx.x < h ? threadIdx.x : nx + threadIdx.x;
        dst[base + i] = src[base + i];
    }
}

hipError_t launch_copy_halo(const void* src, void* dst, int elem_bytes, int64_t nx, int64_t ny, int64_t nz,
                            int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s) {
    const dim3 grid((unsigned)(ny + 2 * h), (unsigned)(nz + 2 * h));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(copy_halo_kernel<double>, grid, dim3(64), 0, s, (const double*)src, (double*)dst, nx,
                           ny, nz, h, pitch_x, pitch_y);
    else
        hipLaunchKernelGGL(copy_halo_kernel<float>, grid, dim3(64), 0, s, (const float*)src, (float*)dst, nx, ny,
                           nz, h, pitch_x, pitch_y);
    return hipGetLastError();
}

// flag <- 1, then flag <- 0 if any halo cell of src has a non-zero bit
// pattern (so -0.0 counts as non-zero).
__global__ void set_flag_kernel(int* flag, int v) { *flag = v; }

template <typename T, typename U>
__global__ void __launch_bounds__(64)
zero_halo_kernel(const T* __restrict__ src, int* flag, int64_t nx, int64_t ny, int64_t nz, int64_t h,
                 int64_t pitch_x, int64_t pitch_y) {
    const int64_t jj = blockIdx.x, kk = blockIdx.y;
    const int64_t base = (kk * pitch_y + jj) * pitch_x;
    const U* s = reinterpret_cast<const U*>(src);
    const bool whole = kk < h || kk >= nz + h || jj < h || jj >= ny + h;
    bool nz_found = false;
    if (whole) {
        for (int64_t i = threadIdx.x; i < nx + 2 * h; i += blockDim.x) nz_found |= s[base + i] != 0;
    } else if (threadIdx.x < 2 * h) {
        const int64_t i = threadIdx.x < h ? threadIdx.x : nx + threadIdx.x;
        nz_found = s[base + i] != 0;
    }
    if (nz_found) *flag = 0;
}

hipError_t launch_zero_halo_flag(const void* src, int* flag, int elem_bytes, int64_t nx, int64_t ny, int64_t nz,
                                 int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, s, flag, 1);
    const dim3 grid((unsigned)(ny + 2 * h), (unsigned)(nz + 2 * h));
    if (elem_bytes == 8)
        hipLaunchKernelGGL((zero_halo_kernel<double, unsigned long long>), grid, dim3(64), 0, s, (const double*)src,
                           flag, nx, ny, nz, h, pitch_x, pitch_y);
    else
        hipLaunchKernelGGL((zero_halo_kernel<float, unsigned int>), grid, dim3(64), 0, s, (const float*)src, flag,
                           nx, ny, nz, h, pitch_x, pitch_y);
    return hipGetLastError();
}

// Partial sums per block: [sum (a-b)^2, sum b^2, max |a-b|, #bitwise-different]
template <typename TA, typename TB>
__global__ void __launch_bounds__(256)
norms_kernel(const TA* __restrict__ a, const TB* __restrict__ b, int64_t nx, int64_t ny, int64_t nz, int64_t h,
             int64_t pitch_x, int64_t pitch_y, double* __restrict__ partial) {
    __shared__ double s_d2[256], s_b2[256], s_mx[256], s_nd[256];
    double d2 = 0, b2 = 0, mx = 0, nd = 0;
    const int64_t total = nx * ny * nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < total;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = n % nx, j = (n / nx) % ny, k = n / (nx * ny);
        const int64_t p = ((k + h) * pitch_y + (j + h)) * pitch_x + (i + h);
        const double av = (double)a[p], bv = (double)b[p];
        const double d = av - bv;
        d2 += d * d;
        b2 += bv * bv;
        const double ad = d < 0 ? -d : d;
        mx = ad > mx || ad != ad ? ad : mx;
        if constexpr (sizeof(TA) == sizeof(TB)) {
            if (sizeof(TA) == 8) {
                nd += __double_as_longlong((double)a[p]) != __double_as_longlong((double)b[p]) ? 1.0 : 0.0;
            } else {
                nd += __float_as_int((float)a[p]) != __float_as_int((float)b[p]) ? 1.0 : 0.0;
            }
        }
    }
    s_d2[threadIdx.x] = d2; s_b2[threadIdx.x] = b2; s_mx[threadIdx.x] = mx; s_nd[threadIdx.x] = nd;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_d2[threadIdx.x] += s_d2[threadIdx.x + w];
            s_b2[threadIdx.x] += s_b2[threadIdx.x + w];
            const double o = s_mx[threadIdx.x + w];
            s_mx[threadIdx.x] = o > s_mx[threadIdx.x] || o != o ? o : s_mx[threadIdx.x];
            s_nd[threadIdx.x] += s_nd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[4 * blockIdx.x + 0] = s_d2[0];
        partial[4 * blockIdx.x + 1] = s_b2[0];
        partial[4 * blockIdx.x + 2] = s_mx[0];
        partial[4 * blockIdx.x + 3] = s_nd[0];
    }
}

hipError_t error_norms(const void* a, int dta, const void* b, int dtb, int64_t nx, int64_t ny, int64_t nz,
                       int64_t h, int64_t pitch_x, int64_t pitch_y, hipStream_t s, double out[4]) {
    const int nblocks = 2048;
    double* partial = nullptr;
    hipError_t e = hipMalloc(&partial, sizeof(double) * 4 * nblocks);
    if (e != hipSuccess) return e;
#define GIRIH_NORMS(TA, TB)                                                                              \
    hipLaunchKernelGGL((norms_kernel<TA, TB>), dim3(nblocks), dim3(256), 0, s, (const TA*)a, (const TB*)b, nx, \
                       ny, nz, h, pitch_x, pitch_y, partial)
    if (dta == DT_F64 && dtb == DT_F64) GIRIH_NORMS(double, double);
    else if (dta == DT_F64) GIRIH_NORMS(double, float);
    else if (dtb == DT_F64) GIRIH_NORMS(float, double);
    else GIRIH_NORMS(float, float);
#undef GIRIH_NORMS
    e = hipGetLastError();
    std::vector<double> host(4 * nblocks);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), partial, sizeof(double) * 4 * nblocks, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(partial);
    if (e != hipSuccess) return e;
    double d2 = 0, b2 = 0, mx = 0, nd = 0;
    for (int i = 0; i < nblocks; ++i) {
        d2 += host[4 * i];
        b2 += host[4 * i + 1];
        const double m = host[4 * i + 2];
        mx = m > mx || m != m ? m : mx;
        nd += host[4 * i + 3];
    }
    out[0] = __builtin_sqrt(d2);
    out[1] = __builtin_sqrt(b2);
    out[2] = mx;
    out[3] = nd;
    return hipSuccess;
}

}  // namespace girih
