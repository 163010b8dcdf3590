// Multi-threaded wavefront diamond (MWD) sweep: one launch per diamond row.
//
// Paper: Section "Approach" (multi-dimensional intra-tile parallelisation,
// the MWD listing and its description), Section "Diamond tiling", Section
// "Wavefront temporal blocking", and the GPU perspective at the end of the
// discussion section.  Mapping onto one CDNA4 compute unit:
//
//  * one workgroup = one extruded diamond (tiled in (t,y)) x one x-chunk;
//    the diamond's intermediate time levels never leave the CU;
//  * the wavefront runs along z: at wavefront step zs, level k of the diamond
//    updates plane zs - R*k (slope R, one plane per step: N_F = 1);
//  * lanes run along x (VX blocks of 64 consecutive cells per lane group), so
//    every global access is a coalesced x-row;
//  * threads split the diamond along y with a fixed data subset per thread
//    at every time level (the paper's fixed-execution-to-data wavefront):
//    each wave owns two y-rows of the diamond, row A at half-distance d from
//    the centre and row B at H-1-d (in blocks of R rows), so every wave
//    updates exactly L = 2H (row, level) cells per step;
//  * each (row, level) cell keeps its last 2R outputs along z in registers
//    (the z-ring): z-neighbours never touch memory.  The centre plane that a
//    level reads from its x- and y-neighbours is staged in LDS once per
//    wavefront step; a barrier separates staging from reading, a second one
//    protects the stage for the next step;
//  * the x-chunk carries a shrinking halo of R*(L-1) cells per side that is
//    recomputed redundantly (the paper keeps x whole on the CPU; on the GPU
//    x is chunked for on-chip capacity and parallel slack).
//
// Register layout: row A may hold any level 1..L-1, row B only levels
// KB_LO..KB_HI (the middle band every partner row lives in), both indexed by
// the level itself, so every ring index and every LDS stage offset except the
// row term is a compile-time constant.
//
// Buffers: diamonds of one row are independent, but redundantly computed
// x-halos read cells that the neighbouring x-chunk of the same diamond may
// already have overwritten under a two-buffer in-place scheme.  Each row
// therefore reads an input pair and writes a separate output pair (four
// arrays in total, alternating per row).  Between rows the state at every y
// is the last two time levels computed there, stored by parity t%2: a diamond
// stores a value iff it does not itself compute the value two levels later,
// and copies the input levels at rows where it computes fewer than two.
#pragma once
#include "stencils.hpp"
#include <type_traits>

namespace girih {

// Compile-time loop: f(std::integral_constant<int, I>) for I = B..E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Opaque copies: the compiler must assume the value changed, so expressions
// derived from it are recomputed where they are used instead of being hoisted
// out of the wavefront loop (which would keep dozens of per-slot scalars and
// lane masks alive across the whole loop and spill them).
__device__ __forceinline__ int opaque_s(int v) {
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ int64_t opaque_s(int64_t v) {
    int lo = opaque_s((int)(uint32_t)(uint64_t)v);
    int hi = opaque_s((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
template <typename T>
__device__ __forceinline__ T opaque_v(T v) { asm volatile("" : "+v"(v)); return v; }

template <typename Real>
struct MwdArgs {
    GridDesc g;
    const Real* in[2];   // input pair, indexed by time parity
    Real* out[2];        // output pair, indexed by time parity
    CoefArgs<Real> coef;
    int64_t T;           // total number of time steps of the run
    int64_t t_c;         // row centre time: row r has t_c = r*H
    int64_t c_first;     // y centre of the diamond with blockIdx.y == 0
    int32_t x_own;       // x cells stored by one workgroup
};

template <int R_, int DW_>
struct DiamondShape {
    static constexpr int R = R_;
    static constexpr int DW = DW_;
    static constexpr int H = DW / (2 * R);
    static constexpr int L = 2 * H;
    // half-width of level k (level k is time step t_c - H + k)
    static constexpr int w(int k) { return k < H ? R * k : DW / 2 - R * (k - H); }
    static constexpr int row_lo(int k) { return DW / 2 - w(k); }
    static constexpr int stage_base(int k) {
        int b = 0;
        for (int q = 0; q < k; ++q) b += 2 * w(q);
        return b;
    }
    // LDS row of (level k, local row j) is stage_row0(k) + j
    static constexpr int stage_row0(int k) { return stage_base(k) - row_lo(k); }
    // levels 0..L-2 are staged (level L-1 feeds no later level of the diamond)
    static constexpr int STAGE_ROWS = stage_base(L - 1) > 0 ? stage_base(L - 1) : 1;
    // the band of levels a partner (row B) can hold
    static constexpr int BMIN = H / 2;
    static constexpr int KB_LO = BMIN + 1;
    static constexpr int KB_HI = L - 1 - BMIN;
    static constexpr int NA = L - 1;
    static constexpr int NB = KB_HI - KB_LO + 1;
    static_assert(DW % (2 * R) == 0, "diamond width must be a multiple of 2R");
    static_assert(R != 1 || H % 2 == 0, "for R = 1 the diamond width must be a multiple of 4");
    static_assert(R == 1 || R % 2 == 0, "row pairing needs an even radius");
};

// Half-distance d (0..DW/2-1) of a row from the diamond centre: the row
// j = DW/2 + d (right) or DW/2 - 1 - d (left).  Its levels are
// [d/R + 1, L - 1 - d/R].  Partner of d: block b = d/R pairs with H-1-b; the
// middle block (H odd) pairs its rows among themselves.
template <class Sh>
__host__ __device__ inline int partner_of(int d) {
    const int b = d / Sh::R, e = d % Sh::R;
    const int b2 = Sh::H - 1 - b;
    return b2 != b ? b2 * Sh::R + e : b * Sh::R + (e ^ 1);
}

// Level range [kf, kl] computed at local row j of a diamond whose local row 0
// is global row y0 (empty: kf > kl).
template <class Sh>
__host__ __device__ inline void row_levels(int j, int64_t y, int64_t ny, int64_t t_c, int64_t T,
                                           int& kf, int& kl) {
    if (j < 0 || j >= Sh::DW || y < 0 || y >= ny) { kf = 1; kl = 0; return; }
    const int d = j >= Sh::DW / 2 ? j - Sh::DW / 2 : Sh::DW / 2 - 1 - j;
    const int b = d / Sh::R;
    int64_t lo = b + 1, hi = Sh::L - 1 - b;
    const int64_t klo = (int64_t)Sh::H - t_c;           // time clip: 0 <= t_c - H + k
    const int64_t khi = T - 1 + Sh::H - t_c;            //            t_c - H + k < T
    if (klo > lo) lo = klo;
    if (khi < hi) hi = khi;
    if (lo > hi) { kf = 1; kl = 0; return; }
    kf = (int)lo; kl = (int)hi;
}

template <class S, typename Real, int DW, int VX>
struct MwdKernel {
    static constexpr int R = S::R;
    using Sh = DiamondShape<R, DW>;
    static constexpr int H = Sh::H, L = Sh::L;
    static constexpr int NWAVES = DW / 2;
    static constexpr int NT = 64 * NWAVES;
    static constexpr int XL = 64 * VX;          // x cells held per row
    static constexpr int HX = R * (L - 1);      // redundant x halo per side
    static constexpr int XOWN_MAX = XL - 2 * HX;
    static constexpr int LDS_BYTES = Sh::STAGE_ROWS * XL * (int)sizeof(Real);
    static constexpr int RING = 2 * R;
    static constexpr int RING_VALUES = (Sh::NA + Sh::NB) * RING * VX;
};

// Per-row state of one wave: the row, its level range, and for r = 1..R bit
// masks over levels k telling whether level k finds its y-neighbour row j-r
// (ym) or j+r (yp) computed at level k-1 inside the diamond (then it reads the
// LDS stage, else the input buffer).
template <int R>
struct RowState {
    int j;
    int64_t y;
    int kf, kl;
    uint32_t ym[R], yp[R];
};

template <class Sh>
__device__ __forceinline__ void init_row(RowState<Sh::R>& rs, int j, int64_t ybase, int64_t ny,
                                         int64_t t_c, int64_t T) {
    rs.j = j;
    rs.y = ybase + j;
    row_levels<Sh>(j, rs.y, ny, t_c, T, rs.kf, rs.kl);
#pragma unroll
    for (int r = 1; r <= Sh::R; ++r) {
        int f, l;
        row_levels<Sh>(j - r, rs.y - r, ny, t_c, T, f, l);
        rs.ym[r - 1] = f <= l ? (((2u << l) - 1u) & ~((1u << f) - 1u)) << 1 : 0u;
        row_levels<Sh>(j + r, rs.y + r, ny, t_c, T, f, l);
        rs.yp[r - 1] = f <= l ? (((2u << l) - 1u) & ~((1u << f) - 1u)) << 1 : 0u;
    }
}

// One (row, level K) cell update for all VX x-blocks of the lane.
//   prev: z-ring of (row, K-1) (valid when K > kf); nvprev: its output this step
//   nv:   output of (row, K) this step (plane zs - R*K)
template <class S, typename Real, int DW, int VX, int K>
__device__ __forceinline__ void update_cell(const MwdArgs<Real>& a, Real* __restrict__ stage,
                                            const RowState<S::R>& rs, const Real (&prev)[2 * S::R][VX],
                                            const Real (&nvprev)[VX], Real (&nv)[VX], int ph, int64_t zs,
                                            int lane, int64_t x0, int ow) {
    using KK = MwdKernel<S, Real, DW, VX>;
    using Sh = typename KK::Sh;
    constexpr int R = S::R, H = Sh::H, L = Sh::L, RING = 2 * R, XL = KK::XL;
    const GridDesc& g = a.g;
#pragma unroll
    for (int v = 0; v < VX; ++v) nv[v] = Real(0);
    const int kf = opaque_s(rs.kf), kl = opaque_s(rs.kl);
    if (K < kf || K > kl) return;
    const int64_t q = opaque_s(zs) - (int64_t)R * K;
    if (q < -R || q >= g.nz + R) return;
    const int64_t s_in = a.t_c - H + K;                 // time level of the inputs
    const Real* __restrict__ src = a.in[s_in & 1];
    const bool from_ring = K > kf;
    const bool q_in = q >= 0 && q < g.nz;
    const bool store_out = K >= kl - 1;
    const bool copy_in = kf == kl;
    const int64_t rowoff = ((q + g.h) * g.pitch_y + (opaque_s(rs.y) + g.h)) * g.pitch_x + g.h;
    lane = opaque_v(lane);
    ow = opaque_s(ow);
    x0 = opaque_s(x0);
    Real* out_new = a.out[(s_in + 1) & 1] + rowoff;
    Real* out_old = a.out[s_in & 1] + rowoff;
    const Real* srow = src + rowoff;
    const int64_t plane = g.plane();
    const int64_t px = g.pitch_x;
    // LDS rows of level K-1: own row, and rows j -/+ r
    const Real* st = stage + (Sh::stage_row0(K - 1 < 0 ? 0 : K - 1) + opaque_s(rs.j)) * XL;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int col = lane + 64 * v;
        const int64_t x = x0 + col;
        const bool x_in = x >= 0 && x < g.nx;
        const bool comp = q_in && x_in && col >= R * K && col < ow + R * (2 * L - 2 - K);
        if (comp) {
            Nbhd<Real, R> n;
            const Real* sp = srow + x;
            if (from_ring) {
                n.c = prev[(ph + R) % RING][v];
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    n.zm[r - 1] = prev[(ph + R - r) % RING][v];
                    n.zp[r - 1] = r == R ? nvprev[v] : prev[(ph + R + r) % RING][v];
                    n.xp[r - 1] = st[col + r];
                    n.xm[r - 1] = st[col - r];
                }
            } else {
                n.c = sp[0];
#pragma unroll
                for (int r = 1; r <= R; ++r) {
                    n.zm[r - 1] = sp[-r * plane];
                    n.zp[r - 1] = sp[r * plane];
                    n.xp[r - 1] = sp[r];
                    n.xm[r - 1] = sp[-r];
                }
            }
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                n.yp[r - 1] = (rs.yp[r - 1] >> K) & 1u ? st[col + r * XL] : sp[r * px];
                n.ym[r - 1] = (rs.ym[r - 1] >> K) & 1u ? st[col - r * XL] : sp[-r * px];
            }
            Real cf[S::NCOEF > 0 ? S::NCOEF : 1];
#pragma unroll
            for (int m = 0; m < S::NCOEF; ++m) cf[m] = a.coef.arr[m][rowoff + x];
            const Real u = S::apply(n, a.coef.k, cf);
            nv[v] = u;
            if (col >= KK::HX && col < KK::HX + ow) {
                if (store_out) out_new[x] = u;
                if (copy_in) out_old[x] = n.c;
            }
        } else if (x >= -R && x < g.nx + R && (!q_in || !x_in)) {
            nv[v] = srow[x];                       // fixed Dirichlet halo (same in every buffer)
        }
    }
}

template <class S, typename Real, int DW, int VX>
__global__ void __launch_bounds__(64 * (DW / 2))
mwd_row_kernel(MwdArgs<Real> a) {
    using KK = MwdKernel<S, Real, DW, VX>;
    using Sh = typename KK::Sh;
    constexpr int R = S::R, L = Sh::L, RING = KK::RING, XL = KK::XL;
    constexpr int NA = Sh::NA, NB = Sh::NB, KB_LO = Sh::KB_LO;
    __shared__ Real stage[Sh::STAGE_ROWS * XL];

    const GridDesc& g = a.g;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int64_t c = a.c_first + (int64_t)blockIdx.y * DW;     // diamond centre (global y)
    const int64_t ybase = c - DW / 2;                           // global y of local row 0
    const int64_t x_own_lo = (int64_t)blockIdx.x * a.x_own;
    const int64_t x_own_hi = x_own_lo + a.x_own < g.nx ? x_own_lo + a.x_own : g.nx;
    const int ow = (int)(x_own_hi - x_own_lo);
    const int64_t x0 = x_own_lo - KK::HX;                       // x of column 0

    // ---- this wave's two rows ------------------------------------------------
    const int per_side = DW / 4;
    const int side = wave / per_side;       // 0: right half (j >= DW/2), 1: left half
    int p = wave % per_side;
    int dA = 0, dB = 0;
    for (int d = 0; d < DW / 2; ++d) {
        const int pd = partner_of<Sh>(d);
        if (d < pd) {
            if (p == 0) { dA = d; dB = pd; }
            --p;
        }
    }
    RowState<R> A, B;
    init_row<Sh>(A, side == 0 ? DW / 2 + dA : DW / 2 - 1 - dA, ybase, g.ny, a.t_c, a.T);
    init_row<Sh>(B, side == 0 ? DW / 2 + dB : DW / 2 - 1 - dB, ybase, g.ny, a.t_c, a.T);

    Real ringA[NA][RING][VX];
    Real ringB[NB][RING][VX];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int m = 0; m < RING; ++m)
#pragma unroll
            for (int v = 0; v < VX; ++v) ringA[i][m][v] = Real(0);
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int m = 0; m < RING; ++m)
#pragma unroll
            for (int v = 0; v < VX; ++v) ringB[i][m][v] = Real(0);

    const int64_t nzs = g.nz + (int64_t)R * (L - 1);   // wavefront steps

    for (int64_t zb = 0; zb < nzs; zb += RING) {
        static_for<0, RING>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t zs = zb + ph;
            const bool live = zs < nzs;          // uniform across the workgroup
            // ---- A: stage the centre planes the next levels read this step ----
            if (live) {
                static_for<0, NA>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int k = 1 + i;
                    if constexpr (k <= L - 2) {
                        const int64_t q = zs - (int64_t)R * (k + 1);
                        if (k >= A.kf && k <= A.kl && q >= 0 && q < g.nz) {
                            Real* st = stage + (Sh::stage_row0(k) + A.j) * XL + lane;
#pragma unroll
                            for (int v = 0; v < VX; ++v) st[64 * v] = ringA[i][(ph + RING - R) % RING][v];
                        }
                    }
                });
                static_for<0, NB>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int k = KB_LO + i;
                    if constexpr (k <= L - 2) {
                        const int64_t q = zs - (int64_t)R * (k + 1);
                        if (k >= B.kf && k <= B.kl && q >= 0 && q < g.nz) {
                            Real* st = stage + (Sh::stage_row0(k) + B.j) * XL + lane;
#pragma unroll
                            for (int v = 0; v < VX; ++v) st[64 * v] = ringB[i][(ph + RING - R) % RING][v];
                        }
                    }
                });
            }
            __syncthreads();
            // ---- B: update every owned (row, level) cell of this step ----------
            if (live) {
                Real nvprev[VX], nv[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) nvprev[v] = Real(0);
                static_for<0, NA>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    update_cell<S, Real, DW, VX, 1 + i>(a, stage, A, ringA[i > 0 ? i - 1 : 0], nvprev, nv,
                                                        ph, zs, lane, x0, ow);
                    if constexpr (i > 0) {
#pragma unroll
                        for (int v = 0; v < VX; ++v) ringA[i - 1][ph][v] = nvprev[v];
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) nvprev[v] = nv[v];
                });
#pragma unroll
                for (int v = 0; v < VX; ++v) ringA[NA - 1][ph][v] = nvprev[v];
#pragma unroll
                for (int v = 0; v < VX; ++v) nvprev[v] = Real(0);
                static_for<0, NB>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    update_cell<S, Real, DW, VX, KB_LO + i>(a, stage, B, ringB[i > 0 ? i - 1 : 0], nvprev, nv,
                                                            ph, zs, lane, x0, ow);
                    if constexpr (i > 0) {
#pragma unroll
                        for (int v = 0; v < VX; ++v) ringB[i - 1][ph][v] = nvprev[v];
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) nvprev[v] = nv[v];
                });
#pragma unroll
                for (int v = 0; v < VX; ++v) ringB[NB - 1][ph][v] = nvprev[v];
                // rows of this diamond with no level in this row: carry both levels
                if (zs < g.nz) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const RowState<R>& rs = t == 0 ? A : B;
                        if (rs.kf > rs.kl && rs.y >= 0 && rs.y < g.ny) {
                            const int64_t rowoff = ((zs + g.h) * g.pitch_y + (rs.y + g.h)) * g.pitch_x + g.h;
#pragma unroll
                            for (int v = 0; v < VX; ++v) {
                                const int col = lane + 64 * v;
                                if (col >= KK::HX && col < KK::HX + ow) {
                                    const int64_t x = x0 + col;
                                    a.out[0][rowoff + x] = a.in[0][rowoff + x];
                                    a.out[1][rowoff + x] = a.in[1][rowoff + x];
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
        });
    }
}

}  // namespace girih
