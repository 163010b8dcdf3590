// Stencil operators of the paper (Listings 1-4) as device functions.
//
// Every kernel in the library (naive sweep and diamond/wavefront sweep) calls
// the same apply() of the same trait, with operands gathered into the same
// named slots, so both schedules execute identical instruction sequences per
// point and agree bit for bit.  The library is compiled with
// -ffp-contract=off: no multiply-add is fused, and the order below is C's
// left-to-right order of the listings.
//
//   Stencil7C  (Listing 1): ((c0*V + c1*(x+ + x-)) + c1*(y+ + y-)) + c1*(z+ + z-)
//   Stencil7V  (Listing 2): C0*V + C1*x+ + C2*x- + C3*y+ + C4*y- + C5*z+ + C6*z-
//   Stencil25C (bracket of Listing 3, first-order Jacobi form):
//              c0*V + c1*S1 + c2*S2 + c3*S3 + c4*S4,
//              S_r = x+r + x-r + y+r + y-r + z+r + z-r   (left to right)
//   Stencil25V (Listing 4): C00*V + C01*(x+1 + x-1) + C02*(y+1 + y-1)
//              + C03*(z+1 + z-1) + ... + C12*(z+4 + z-4)
//   Stencil25L (Listing 3 as printed, second order in time):
//              (2*V - Uold) + C*(c0*V + c1*S1 + c2*S2 + c3*S3 + c4*S4),
//              Uold = the point's value at time t-1 (the array being written)
//   Stencil27B (the 27-point box stencil of Section "Handling other stencil
//              types"; the paper gives no listing, so the order is the
//              library's): ((c0*V + c1*F) + c2*E) + c3*K, F / E / K the sums of
//              the 6 face, 12 edge and 8 corner neighbours, each in
//              lexicographic order of the offset (dz, dy, dx), -1 < 0 < +1
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace girih {

// Neighbourhood of one point: centre, and for r = 1..R the six axis
// neighbours; uo is the point's previous value (second-order-in-time stencils
// only; LEAPFROG says whether a stencil reads it).  BOX: the stencil reads
// the whole 3x3x3 box (Box27 below) instead.
template <typename Real, int R>
struct Nbhd {
    Real c;
    Real xp[R], xm[R], yp[R], ym[R], zp[R], zm[R];
    Real uo;
};

struct Stencil7C {
    static constexpr int R = 1, NCOEF = 0, NCONST = 2;
    static constexpr bool LEAPFROG = false;
    static constexpr bool BOX = false;
    template <typename Real>
    __device__ __forceinline__ static Real apply(const Nbhd<Real, 1>& n, const Real* k, const Real*) {
        return ((k[0] * n.c + k[1] * (n.xp[0] + n.xm[0])) + k[1] * (n.yp[0] + n.ym[0]))
               + k[1] * (n.zp[0] + n.zm[0]);
    }
};

struct Stencil7V {
    static constexpr int R = 1, NCOEF = 7, NCONST = 0;
    static constexpr bool LEAPFROG = false;
    static constexpr bool BOX = false;
    template <typename Real>
    __device__ __forceinline__ static Real apply(const Nbhd<Real, 1>& n, const Real*, const Real* C) {
        Real u = C[0] * n.c;
        u = u + C[1] * n.xp[0];
        u = u + C[2] * n.xm[0];
        u = u + C[3] * n.yp[0];
        u = u + C[4] * n.ym[0];
        u = u + C[5] * n.zp[0];
        u = u + C[6] * n.zm[0];
        return u;
    }
};

struct Stencil25C {
    static constexpr int R = 4, NCOEF = 0, NCONST = 5;
    static constexpr bool LEAPFROG = false;
    static constexpr bool BOX = false;
    template <typename Real>
    __device__ __forceinline__ static Real apply(const Nbhd<Real, 4>& n, const Real* k, const Real*) {
        Real u = k[0] * n.c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Real s = n.xp[r] + n.xm[r];
            s = s + n.yp[r];
            s = s + n.ym[r];
            s = s + n.zp[r];
            s = s + n.zm[r];
            u = u + k[r + 1] * s;
        }
        return u;
    }
};

struct Stencil25V {
    static constexpr int R = 4, NCOEF = 13, NCONST = 0;
    static constexpr bool LEAPFROG = false;
    static constexpr bool BOX = false;
    template <typename Real>
    __device__ __forceinline__ static Real apply(const Nbhd<Real, 4>& n, const Real*, const Real* C) {
        Real u = C[0] * n.c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            u = u + C[3 * r + 1] * (n.xp[r] + n.xm[r]);
            u = u + C[3 * r + 2] * (n.yp[r] + n.ym[r]);
            u = u + C[3 * r + 3] * (n.zp[r] + n.zm[r]);
        }
        return u;
    }
};

struct Stencil25L {
    static constexpr int R = 4, NCOEF = 1, NCONST = 5;
    static constexpr bool LEAPFROG = true;
    static constexpr bool BOX = false;
    template <typename Real>
    __device__ __forceinline__ static Real apply(const Nbhd<Real, 4>& n, const Real* k, const Real* C) {
        Real b = k[0] * n.c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Real s = n.xp[r] + n.xm[r];
            s = s + n.yp[r];
            s = s + n.ym[r];
            s = s + n.zp[r];
            s = s + n.zm[r];
            b = b + k[r + 1] * s;
        }
        return (Real(2) * n.c - n.uo) + C[0] * b;
    }
};

// The 3x3x3 neighbourhood of a point, v[(dz+1)*9 + (dy+1)*3 + (dx+1)].
template <typename Real>
struct Box27 {
    Real v[27];
};

struct Stencil27B {
    static constexpr int R = 1, NCOEF = 0, NCONST = 4;
    static constexpr bool LEAPFROG = false;
    static constexpr bool BOX = true;
    template <typename Real>
    __device__ __forceinline__ static Real apply_box(const Box27<Real>& b, const Real* k) {
        // class of offset m: number of nonzero components (compile-time)
        Real f = b.v[4], e = b.v[1], q = b.v[0];   // first face (-1,0,0), edge (-1,-1,0), corner (-1,-1,-1)
#pragma unroll
        for (int m = 2; m < 27; ++m) {
            const int cls = (m / 9 != 1) + ((m / 3) % 3 != 1) + (m % 3 != 1);
            if (m == 4) continue;
            if (cls == 1) f = f + b.v[m];
            else if (cls == 2 && m != 1) e = e + b.v[m];
        }
#pragma unroll
        for (int m = 1; m < 27; ++m) {
            const int cls = (m / 9 != 1) + ((m / 3) % 3 != 1) + (m % 3 != 1);
            if (cls == 3) q = q + b.v[m];
        }
        return ((k[0] * b.v[13] + k[1] * f) + k[2] * e) + k[3] * q;
    }
};

// Grid geometry shared by all kernels: element (k,j,i), k in [-h,nz+h) etc.,
// is at ((k+h)*pitch_y + (j+h))*pitch_x + (i+h).
struct GridDesc {
    int64_t nx, ny, nz;
    int64_t pitch_x, pitch_y;
    int32_t h;
    __host__ __device__ __forceinline__ int64_t idx(int64_t k, int64_t j, int64_t i) const {
        return ((k + h) * pitch_y + (j + h)) * pitch_x + (i + h);
    }
    __host__ __device__ __forceinline__ int64_t plane() const { return pitch_y * pitch_x; }
};

// Up to 13 coefficient arrays and 5 constants, passed by value.
template <typename Real>
struct CoefArgs {
    const Real* arr[13];
    Real k[5];
};

}  // namespace girih
