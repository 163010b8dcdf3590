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
//  * lanes run along x (VX blocks of 64 consecutive cells), so every global
//    access is a coalesced x-row;
//  * threads split the diamond along y with a fixed data subset per thread
//    at every time level (the paper's fixed-execution-to-data wavefront):
//    each wave owns two y-rows of the diamond, row A at half-distance d from
//    the centre and row B at H-1-d (in blocks of R rows), so every wave
//    updates exactly L = 2H (row, level) cells per step;
//  * each (row, level) cell keeps its last 2R outputs along z in registers
//    (the z-ring): z-neighbours never touch memory;
//  * the plane each level reads its x- and y-neighbours from is staged in
//    LDS once per wavefront step: computed levels from their z-rings, and the
//    cells of the previous diamond row a level needs (its entry inputs and
//    the rows just outside it) from HBM, loaded one step ahead into
//    registers so no HBM latency sits between two barriers;
//  * a row's first computed level takes its z-neighbours from a "virtual"
//    z-ring of the input time level, fed by the same one-step-ahead loads;
//  * the x-chunk carries a shrinking halo of R*(L-1) cells per side that is
//    recomputed redundantly (the paper keeps x whole on the CPU; on the GPU x
//    is chunked for on-chip capacity and parallel slack); all lanes compute
//    every cell, values outside a level's valid range are never consumed.
//
// Register layout: row A may hold any level 1..L-1, row B only levels
// KB_LO..KB_HI (the band every partner row lives in), both indexed by the
// level itself, so every ring index and every LDS offset except the row term
// is a compile-time constant.
//
// Buffers: diamonds of one row are independent, but redundantly computed
// x-halos read cells that the neighbouring x-chunk of the same diamond may
// already have overwritten under a two-buffer in-place scheme.  Each row
// therefore reads an input pair and writes a separate output pair (four
// arrays in total, alternating per row).  Between rows the state at every y
// is the last two time levels computed there, stored by parity t%2: a diamond
// stores a value iff it does not itself compute the value two levels later,
// and copies the input levels at rows where it computes fewer than two.
//
// Dirichlet halo: if the halo of the input is all zero (a flag computed on
// the device before the sweep) halo rows of the stage are zero-filled once
// and halo lanes and planes are set to zero; otherwise halo values are loaded
// where they are needed (slower, same result).
#pragma once
#include <type_traits>

#include "stencils.hpp"

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
// out of the wavefront loop (which would keep dozens of per-slot scalars
// alive across the loop and spill them).
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

template <typename Real>
struct MwdArgs {
    GridDesc g;
    const Real* in[2];   // input pair, indexed by time parity
    Real* out[2];        // output pair, indexed by time parity
    CoefArgs<Real> coef;
    const int* zero_halo;  // device flag: 1 if every halo cell of the input is zero
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
    // stage level k (0..L-2) holds the rows level k+1 reads: Y_{k+1} +- R
    static constexpr int sl_lo(int k) { return DW / 2 - w(k + 1) - R; }
    static constexpr int nrows(int k) { return 2 * w(k + 1) + 2 * R; }
    static constexpr int sbase(int k) {
        int b = 0;
        for (int q = 0; q < k; ++q) b += nrows(q);
        return b;
    }
    // LDS row of (stage level k, local row j) is srow0(k) + j
    static constexpr int srow0(int k) { return sbase(k) - sl_lo(k); }
    static constexpr int STAGE_ROWS = sbase(L - 1);
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

// Level range [kf, kl] computed at local row j whose global row is y
// (empty: kf > kl).
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
    static constexpr int XLP = XL + 2 * R;      // LDS row stride (R guard cells per side)
    static constexpr int HX = R * (L - 1);      // redundant x halo per side
    static constexpr int XOWN_MAX = XL - 2 * HX;
    static constexpr int LDS_BYTES = Sh::STAGE_ROWS * XLP * (int)sizeof(Real);
    static constexpr int RING = 2 * R;
};

// One-step-ahead registers of an owned row: the cells of earlier diamond rows
// it needs.
template <typename Real, int VX>
struct RowRegs {
    Real vnext[VX];          // input level kf-1: plane it "produces" at the coming step
    Real pre1[VX];           // stage duty kv of a row that computes nothing here
    Real pre2[VX];           // stage duty kv-1
    Real preo[VX];           // out-of-span neighbour row for the coming step's stage
};

// Stage duties of one owned row.  Level k of the stage holds the time level
// t_c-H+k+1 that level k+1 reads.  A row's cells not computed in this diamond
// but read by its neighbours are the (at most two) levels just below its first
// computed level -- or, for a row the end of the run leaves empty, below the
// level it would have entered at -- and they come from the input pair.  A row
// that computes keeps level kf-1 in the slot of that level (its input ring),
// fed by the one-step-ahead loads, and stages it like a computed level.
struct RowDuty {
    int kv;        // upper duty level (kf-1 when the row computes)
    bool d1, d2;   // stage kv from a prefetch register (rows that compute nothing), stage kv-1
};

// byte-offset access: uniform row pointer + per-lane 32-bit byte offset
template <typename Real>
__device__ __forceinline__ Real ld_at(const Real* row, uint32_t byte_off) {
    return *reinterpret_cast<const Real*>(reinterpret_cast<const char*>(row) + byte_off);
}
template <typename Real>
__device__ __forceinline__ void st_at(Real* row, uint32_t byte_off, Real v) {
    *reinterpret_cast<Real*>(reinterpret_cast<char*>(row) + byte_off) = v;
}

template <class S, typename Real, int DW, int VX>
__global__ void __launch_bounds__(64 * (DW / 2))
mwd_row_kernel(MwdArgs<Real> a) {
    using KK = MwdKernel<S, Real, DW, VX>;
    using Sh = typename KK::Sh;
    constexpr int R = S::R, H = Sh::H, L = Sh::L, RING = KK::RING, XLP = KK::XLP;
    constexpr int KB0 = Sh::KB_LO - 1;            // first slot level of row B
    constexpr int NA = L;                         // row A slots: levels 0..L-1
    constexpr int NB = Sh::KB_HI - KB0 + 1;       // row B slots: levels KB0..KB_HI
    __shared__ Real stage[Sh::STAGE_ROWS * XLP];

    const GridDesc& g = a.g;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int64_t c = a.c_first + (int64_t)blockIdx.y * DW;     // diamond centre (global y)
    const int64_t ybase = c - DW / 2;                           // global y of local row 0
    const int64_t x_own_lo = (int64_t)blockIdx.x * a.x_own;
    const int64_t x_own_hi = x_own_lo + a.x_own < g.nx ? x_own_lo + a.x_own : g.nx;
    const int64_t x0 = x_own_lo - KK::HX;                       // x of column 0
    const int zero_halo = __builtin_amdgcn_readfirstlane(*a.zero_halo);
    const bool edge_x = x0 < 0 || x0 + KK::XL > g.nx;          // chunk touches the x halo
    const bool edge_y = ybase - R < 0 || ybase + DW + R > g.ny; // diamond touches the y halo

    // per-lane constants: clamped byte offset within a row, ownership, x-halo
    uint32_t xb[VX];
    bool own[VX], xh[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int64_t x = x0 + lane + 64 * v;
        const int64_t xc = x < -R ? -R : (x >= g.nx + R ? g.nx + R - 1 : x);
        xb[v] = (uint32_t)((xc + g.h) * (int64_t)sizeof(Real));
        own[v] = x >= x_own_lo && x < x_own_hi;
        xh[v] = (x >= -R && x < 0) || (x >= g.nx && x < g.nx + R);
    }

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
    const int jA = side == 0 ? DW / 2 + dA : DW / 2 - 1 - dA;
    const int jB = side == 0 ? DW / 2 + dB : DW / 2 - 1 - dB;
    int kfA, klA, kfB, klB;
    row_levels<Sh>(jA, ybase + jA, g.ny, a.t_c, a.T, kfA, klA);
    row_levels<Sh>(jB, ybase + jB, g.ny, a.t_c, a.T, kfB, klB);
    auto in_layout = [&](int k, int j) -> bool {
        if (k < 0 || k > L - 2) return false;
        const int wk = (k + 1) < H ? R * (k + 1) : DW / 2 - R * (k + 1 - H);
        return j >= DW / 2 - wk - R && j < DW / 2 + wk + R;
    };
    auto duty_of = [&](int d, int j, int kf, int kl) -> RowDuty {
        RowDuty du{-1, false, false};
        const int64_t y = ybase + j;
        if (y < 0 || y >= g.ny) return du;
        const int64_t kmax64 = a.T - 1 + H - a.t_c;   // last level inside the run
        const int kmax = kmax64 > L - 1 ? L - 1 : (int)kmax64;
        const int ks = d / R + 1;                      // level the diamond shape enters at
        du.kv = kf <= kl ? kf - 1 : (ks - 1 < kmax - 1 ? ks - 1 : kmax - 1);
        auto ok = [&](int k) { return k >= 0 && a.t_c - H + k + 1 >= 0 && in_layout(k, j); };
        du.d1 = kf > kl && ok(du.kv);
        du.d2 = ok(du.kv - 1);
        return du;
    };
    const RowDuty uA = duty_of(dA, jA, kfA, klA);
    const RowDuty uB = duty_of(dB, jB, kfB, klB);
    // level bit masks of each row: computed, stored (last two computed), input copied
    auto bits = [](int lo, int hi) -> uint32_t {
        return lo > hi ? 0u : (((2u << hi) - 1u) & ~((1u << lo) - 1u));
    };
    const uint32_t cmaskA = bits(kfA, klA), cmaskB = bits(kfB, klB);
    const uint32_t smaskA = bits(kfA > klA - 1 ? kfA : klA - 1, klA);
    const uint32_t smaskB = bits(kfB > klB - 1 ? kfB : klB - 1, klB);
    const uint32_t cpmaskA = kfA == klA ? cmaskA : 0u, cpmaskB = kfB == klB ? cmaskB : 0u;
    // byte offset of row y within a plane (rows of computing slots are inside the grid)
    const int rowbA = (int)((ybase + jA + g.h) * g.pitch_x * (int64_t)sizeof(Real));
    const int rowbB = (int)((ybase + jB + g.h) * g.pitch_x * (int64_t)sizeof(Real));
    // The outermost block of rows reads, at level H, the rows up to R beyond
    // the diamond at level H-1 (time t_c).  The owner of an outermost row j
    // stages the row R further out (j+R on the right, j-R on the left); it does
    // so whether or not its own row is inside the grid.
    auto out_row = [&](int d, int j) -> int {
        if (d / R != H - 1 || a.t_c >= a.T) return -1000;
        const int jo = side == 0 ? j + R : j - R;
        const int64_t yo = ybase + jo;
        return yo >= -R && yo < g.ny + R ? jo : -1000;
    };
    const int joA = out_row(dA, jA);
    const int joB = out_row(dB, jB);

    const int64_t plane = g.plane();
    // element offset of (plane q, global row y); q clamped into the haloed box
    auto rowoff = [&](int64_t q, int64_t y) -> int64_t {
        q = q < -R ? -R : (q >= g.nz + R ? g.nz + R - 1 : q);
        return (q + g.h) * plane + (y + g.h) * g.pitch_x;
    };
    auto srow = [&](int k, int j) -> Real* { return stage + (Sh::srow0(k) + j) * XLP + R; };
    auto load_row = [&](const Real* base, int64_t off, Real (&dst)[VX]) {
        const Real* rp = base + off;
#pragma unroll
        for (int v = 0; v < VX; ++v) dst[v] = ld_at(rp, xb[v]);
    };
    // Stage a row; with a zero halo the x-halo columns are written as zero here
    // (their register values are never fixed up on that path).
    auto put_row = [&](Real* sp, const Real (&src)[VX]) {
        if (edge_x && zero_halo) {
#pragma unroll
            for (int v = 0; v < VX; ++v) sp[lane + 64 * v] = xh[v] ? Real(0) : src[v];
        } else {
#pragma unroll
            for (int v = 0; v < VX; ++v) sp[lane + 64 * v] = src[v];
        }
    };

    // Halo rows of the stage (rows outside the grid, inside it +-R): with a zero
    // halo they are written once here and never touched again.
    if (edge_y && zero_halo) {
        for (int k = 0; k < L - 1; ++k) {
            for (int j = Sh::sl_lo(k); j < Sh::sl_lo(k) + Sh::nrows(k); ++j) {
                const int64_t y = ybase + j;
                if ((y >= -R && y < 0) || (y >= g.ny && y < g.ny + R)) {
                    Real* sp = srow(k, j) - R;
                    for (int col = threadIdx.x; col < XLP; col += KK::NT) sp[col] = Real(0);
                }
            }
        }
    }

    // z-rings: ring[i][m] holds the output of slot i (level K0 + i) at the last
    // 2R wavefront steps, entry m for steps congruent to m mod 2R.
    Real ringA[NA][RING][VX];
    Real ringB[NB][RING][VX];
    RowRegs<Real, VX> RA, RB;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        RA.vnext[v] = RA.pre1[v] = RA.pre2[v] = RA.preo[v] = Real(0);
        RB.vnext[v] = RB.pre1[v] = RB.pre2[v] = RB.preo[v] = Real(0);
    }
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

    // One-step-ahead loads of a row for step `zs`: the input level kf-1 at the
    // plane it "produces" at that step, and the stage rows of that step.
    auto prefetch = [&](RowRegs<Real, VX>& rr, int j, int kf, int kl, const RowDuty& du, int jo, int64_t zs) {
        if (jo > -1000) load_row(a.in[a.t_c & 1], rowoff(zs - (int64_t)R * H, ybase + jo), rr.preo);
        const int64_t y = ybase + j;
        const int64_t tv = a.t_c - H + du.kv + 1;   // time level of stage duty kv
        if (kf <= kl) load_row(a.in[tv & 1], rowoff(zs - (int64_t)R * du.kv, y), rr.vnext);
        if (du.d1) load_row(a.in[tv & 1], rowoff(zs - (int64_t)R * (du.kv + 1), y), rr.pre1);
        if (du.d2) load_row(a.in[(tv - 1) & 1], rowoff(zs - (int64_t)R * du.kv, y), rr.pre2);
    };

    // The sweep starts 2R steps early so that the input rings of rows entering
    // at level 1 hold the halo planes -R..-1; steps before 0 compute nothing.
    prefetch(RA, jA, kfA, klA, uA, joA, -RING);
    prefetch(RB, jB, kfB, klB, uB, joB, -RING);
    __syncthreads();

    const int64_t nzs = g.nz + (int64_t)R * (L - 1);   // wavefront steps end here

    for (int64_t zb = -RING; zb < nzs; zb += RING) {
        static_for<0, RING>([&](auto phc) {
            constexpr int ph = decltype(phc)::value;
            const int64_t zs = zb + ph;
            const bool live = zs < nzs;          // uniform across the workgroup
            Real vcurA[VX], vcurB[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) { vcurA[v] = RA.vnext[v]; vcurB[v] = RB.vnext[v]; }
            // ---- A: stage every plane the levels read this step ------------------
            if (live) {
                const int kfa = opaque_s(kfA), kla = opaque_s(klA), kfb = opaque_s(kfB), klb = opaque_s(klB);
                const int ja = opaque_s(jA), jb = opaque_s(jB);
                // computed levels and the input level kf-1 of rows that compute
                static_for<0, NA>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int k = i;
                    if constexpr (k <= L - 2) {
                        if (k >= kfa - 1 && k <= kla) put_row(srow(k, ja), ringA[i][(ph + RING - R) % RING]);
                    }
                });
                static_for<0, NB>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int k = KB0 + i;
                    if constexpr (k <= L - 2) {
                        if (k >= kfb - 1 && k <= klb) put_row(srow(k, jb), ringB[i][(ph + RING - R) % RING]);
                    }
                });
                auto stage_row = [&](RowRegs<Real, VX>& rr, int j, const RowDuty& du, int jo) {
                    if (jo > -1000) put_row(srow(H - 1, jo), rr.preo);
                    if (du.d1) put_row(srow(du.kv, j), rr.pre1);
                    if (du.d2) put_row(srow(du.kv - 1, j), rr.pre2);
                };
                stage_row(RA, ja, uA, opaque_s(joA));
                stage_row(RB, jb, uB, opaque_s(joB));
                // halo rows with a non-zero halo: load them (latency exposed; edge diamonds only)
                if (edge_y && !zero_halo) {
                    for (int k = wave; k < L - 1; k += KK::NWAVES) {
                        for (int j = Sh::sl_lo(k); j < Sh::sl_lo(k) + Sh::nrows(k); ++j) {
                            const int64_t y = ybase + j;
                            if ((y >= -R && y < 0) || (y >= g.ny && y < g.ny + R)) {
                                Real tmp[VX];
                                load_row(a.in[0], rowoff(zs - (int64_t)R * (k + 1), y), tmp);
                                put_row(srow(k, j), tmp);
                            }
                        }
                    }
                }
                // loads for the next step
                prefetch(RA, ja, kfa, kla, uA, opaque_s(joA), zs + 1);
                prefetch(RB, jb, kfb, klb, uB, opaque_s(joB), zs + 1);
            }
            __syncthreads();
            // ---- B: update every owned (row, level) cell of this step ----------
            if (live) {
                // Addresses: every plane a computing slot touches lies in the window
                // [zs - R*L, zs]; a uniform 64-bit window base per array plus a
                // 32-bit byte offset (per slot uniform + per lane) reaches it.
                // The parity of level K's input time level t_c-H+K is p0 ^ (K & 1).
                const int64_t e0 = (zs - (int64_t)R * L + g.h) * plane;
                const int p0 = (int)((a.t_c - H) & 1);
                const Real* in_par[2] = {a.in[p0] + e0, a.in[p0 ^ 1] + e0};
                Real* out_par[2] = {a.out[p0] + e0, a.out[p0 ^ 1] + e0};
                const uint32_t plane_b = (uint32_t)(plane * (int64_t)sizeof(Real));
                // levels whose plane zs - R*K is inside the grid
                const int64_t khz = zs >= 0 ? zs / R : -1;
                const int64_t klz = zs - g.nz >= 0 ? (zs - g.nz) / R + 1 : 0;
                const uint32_t zmask = khz < klz ? 0u
                    : ((khz >= 31 ? 0xffffffffu : ((2u << khz) - 1u)) & ~((1u << (klz > 31 ? 31 : klz)) - 1u));
                // One slot of one row: levels kf..kl compute, every other slot
                // passes the loaded input plane on (the input level kf-1 keeps it
                // in its ring).  prev is the slot below's output at this step (the
                // z+R neighbour); the slot below's ring is updated only after this
                // slot has read it.
                auto slot = [&](auto ic, auto k0c, auto& ring, Real (&prev)[VX], const Real (&vcur)[VX],
                                const Real* st_row, uint32_t rowb, uint32_t cmask, uint32_t smask,
                                uint32_t cpmask, int64_t y) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int K = decltype(k0c)::value + i;
                    constexpr int KP = K & 1;
                    Real nv[VX];
#pragma unroll
                    for (int v = 0; v < VX; ++v) nv[v] = vcur[v];
                    if constexpr (i > 0) {
                        if ((cmask >> K) & 1u) {
                            if ((zmask >> K) & 1u) {
                                const uint32_t so = (uint32_t)(R * (L - K)) * plane_b + rowb;
                                const Real* st = st_row + Sh::srow0(K - 1) * XLP;
                                const bool cpy = (cpmask >> K) & 1u;
                                Real cin[VX];
#pragma unroll
                                for (int v = 0; v < VX; ++v) {
                                    const int col = lane + 64 * v;
                                    const uint32_t vo = so + xb[v];
                                    Nbhd<Real, R> n;
                                    n.c = ring[i - 1][(ph + R) % RING][v];
#pragma unroll
                                    for (int r = 1; r <= R; ++r) {
                                        n.zm[r - 1] = ring[i - 1][(ph + R - r) % RING][v];
                                        n.zp[r - 1] = r == R ? prev[v] : ring[i - 1][(ph + R + r) % RING][v];
                                        n.xp[r - 1] = st[col + r];
                                        n.xm[r - 1] = st[col - r];
                                        n.yp[r - 1] = st[col + r * XLP];
                                        n.ym[r - 1] = st[col - r * XLP];
                                    }
                                    Real cf[S::NCOEF > 0 ? S::NCOEF : 1];
#pragma unroll
                                    for (int m = 0; m < S::NCOEF; ++m) cf[m] = ld_at(a.coef.arr[m] + e0, vo);
                                    nv[v] = S::apply(n, a.coef.k, cf);
                                    if (cpy) cin[v] = n.c;
                                }
                                // x-halo lanes hold the fixed halo (a zero halo is
                                // written into the stage instead, see put_row)
                                if (edge_x && !zero_halo) {
#pragma unroll
                                    for (int v = 0; v < VX; ++v)
                                        if (xh[v]) nv[v] = ld_at(in_par[0], so + xb[v]);
                                }
                                // the last two levels of a row go to the output pair
                                if ((smask >> K) & 1u) {
#pragma unroll
                                    for (int v = 0; v < VX; ++v)
                                        if (own[v]) st_at(out_par[KP ^ 1], so + xb[v], nv[v]);
                                }
                                if (cpy) {
#pragma unroll
                                    for (int v = 0; v < VX; ++v)
                                        if (own[v]) st_at(out_par[KP], so + xb[v], cin[v]);
                                }
                            } else {
#pragma unroll
                                for (int v = 0; v < VX; ++v) nv[v] = Real(0);
                                const int64_t q = zs - (int64_t)R * K;
                                if (!zero_halo && q >= -R && q < g.nz + R)
                                    load_row(a.in[0], rowoff(q, y), nv);   // fixed halo plane
                            }
                        }
#pragma unroll
                        for (int v = 0; v < VX; ++v) ring[i - 1][ph][v] = prev[v];
                    }
#pragma unroll
                    for (int v = 0; v < VX; ++v) prev[v] = nv[v];
                };
                Real prevA[VX], prevB[VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) { prevA[v] = vcurA[v]; prevB[v] = vcurB[v]; }
                const Real* stA = stage + opaque_s(jA) * XLP + R;
                const Real* stB = stage + opaque_s(jB) * XLP + R;
                const uint32_t rbA = (uint32_t)opaque_s(rowbA), rbB = (uint32_t)opaque_s(rowbB);
                const uint32_t cmA = (uint32_t)opaque_s((int)cmaskA), cmB = (uint32_t)opaque_s((int)cmaskB);
                const uint32_t smA = (uint32_t)opaque_s((int)smaskA), smB = (uint32_t)opaque_s((int)smaskB);
                const uint32_t cpA = (uint32_t)opaque_s((int)cpmaskA), cpB = (uint32_t)opaque_s((int)cpmaskB);
                // interleave the two rows level by level: two independent chains
                static_for<0, NA>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    slot(ic, std::integral_constant<int, 0>{}, ringA, prevA, vcurA, stA, rbA, cmA, smA, cpA,
                         ybase + jA);
                    if constexpr (i >= KB0 && i - KB0 < NB) {
                        slot(std::integral_constant<int, i - KB0>{}, std::integral_constant<int, KB0>{}, ringB, prevB,
                             vcurB, stB, rbB, cmB, smB, cpB, ybase + jB);
                    }
                });
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    ringA[NA - 1][ph][v] = prevA[v];
                    ringB[NB - 1][ph][v] = prevB[v];
                }
                // rows of this diamond with no level in this row: carry both levels
                if (zs >= 0 && zs < g.nz) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int jr = t == 0 ? jA : jB;
                        const int kf = t == 0 ? kfA : kfB, kl = t == 0 ? klA : klB;
                        const int64_t y = ybase + jr;
                        if (kf > kl && y >= 0 && y < g.ny) {
                            const int64_t ro = rowoff(zs, y);
#pragma unroll
                            for (int v = 0; v < VX; ++v) {
                                if (own[v]) {
                                    st_at(a.out[0] + ro, xb[v], ld_at(a.in[0] + ro, xb[v]));
                                    st_at(a.out[1] + ro, xb[v], ld_at(a.in[1] + ro, xb[v]));
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
