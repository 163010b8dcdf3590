// Multi-threaded wavefront diamond (MWD) sweep: one launch per diamond row
// (mwd_row_kernel), or one launch of every row's tiles in dependency order
// (mwd_sweep_kernel, further below).
//
// Paper: Section "Approach" (multi-dimensional intra-tile parallelisation,
// the MWD listing and its description), Section "Diamond tiling", Section
// "Wavefront temporal blocking", and the GPU perspective at the end of the
// discussion section.  Mapping onto one CDNA4 compute unit:
//
//  * one workgroup = one extruded diamond (tiled in (t,y)) x one x-chunk;
//    the diamond's intermediate time levels never leave the CU;
//  * the wavefront runs along z in steps of NF planes (the wavefront depth
//    N_F): a step advances one slab of NF consecutive planes, and at step zs
//    level k of the diamond updates slab zs - RZ*k, RZ = ceil(R/NF) slabs
//    (the paper skews the levels by R planes; a level here also takes its
//    x/y neighbours of the slab from the level below's previous steps, so the
//    skew is at least one slab);
//  * lanes run along x (VX blocks of 64 consecutive cells), so every global
//    access is a coalesced x-row;
//  * threads split the diamond along y with a fixed data subset per thread
//    at every time level (the paper's fixed-execution-to-data wavefront):
//    each wave owns two y-rows of the diamond, row A at half-distance d from
//    the centre and row B at H-1-d (in blocks of R rows), so every wave
//    updates exactly L = 2H (row, level) cells per step;
//  * each (row, level) cell keeps its last 2*RZ slabs along z in registers
//    (the z-ring): z-neighbours never touch memory;
//  * the slab each level reads its x- and y-neighbours from is staged in
//    LDS once per wavefront step (NF sub-rows per stage row): computed
//    levels from their z-rings, and the cells of the previous diamond row a
//    level needs (its entry inputs and the rows just outside it) from HBM,
//    loaded one step ahead into registers so no HBM latency sits between
//    two barriers;
//  * a row's first computed level takes its z-neighbours from a "virtual"
//    z-ring of the input time level, fed by the same one-step-ahead loads;
//  * the x-chunk carries a shrinking halo of R*(L-1) cells per side that is
//    recomputed redundantly (the paper keeps x whole on the CPU; on the GPU x
//    is chunked for on-chip capacity and parallel slack); all lanes compute
//    every cell, values outside a level's valid range are never consumed.
//
// Register layout: a wave's two rows form one list of register slots (row
// A's input level and computed levels, then row B's), so every wave runs the
// same code whatever its rows' level ranges; a slot's ring sits at a
// compile-time register index, its level and LDS row are per-wave values.
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
// the device before the sweep) the halo rows and the x-halo columns of the
// stage are zero-filled once (halo lanes never write the stage) and halo
// planes are set to zero; otherwise halo values are loaded where they are
// needed (slower, same result).
//
// Within a wavefront step the waves synchronise with workgroup barriers, or
// (SY = 1) wait only for the waves they share stage rows with.  Stencils
// with coefficient arrays load a slot's coefficients with its neighbours;
// the second-order-in-time stencil also reads, for each level, the level two
// below at its own cell (mwd_tile).
#pragma once
#include <type_traits>

#include "lanes.hpp"
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
    int64_t c_first;     // y centre of the row's first diamond
    int32_t x_own;       // x cells stored by one workgroup
    // relaxed synchronisation within a tile: a wait on the waves of the
    // workgroup gives up after spin_limit polls and sets *error (nonzero)
    uint32_t* error;
    uint32_t spin_limit;
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
    // levels 0..L-2 (read by the level above) and level L-1, whose 2R rows are
    // staged only to be stored
    static constexpr int STAGE_ROWS = sbase(L);
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

// The two rows of row pair pw (0 .. DW/2-1): pairs 0 .. DW/4-1 take the
// right half of the diamond (j >= DW/2), the others the left half; within a
// half, pair p takes the p-th half-distance d (in increasing order) that is
// smaller than its partner, and that partner.
template <class Sh>
__host__ __device__ inline void pair_rows(int pw, int& dA, int& dB, int& jA, int& jB) {
    const int per_side = Sh::DW / 4;
    const int side = pw / per_side;   // 0: right half, 1: left half
    int p = pw % per_side;
    dA = dB = 0;
    for (int d = 0; d < Sh::DW / 2; ++d) {
        const int pd = partner_of<Sh>(d);
        if (d < pd) {
            if (p == 0) { dA = d; dB = pd; }
            --p;
        }
    }
    jA = side == 0 ? Sh::DW / 2 + dA : Sh::DW / 2 - 1 - dA;
    jB = side == 0 ? Sh::DW / 2 + dB : Sh::DW / 2 - 1 - dB;
}

// Waves of a workgroup whose stage rows a wave of row pair pw reads, or which
// read its stage rows (level k+1 of a row reads level k of the rows within R
// of it; a wave stages its two rows and, for a row in the outermost block of
// R rows, the row R beyond it), plus the waves of the same row pair (other x
// slices, whose edge cells it reads): one bit per wave w, pair w % npairs.
template <class Sh>
__host__ __device__ inline uint32_t pair_neighbours(int pw, int npairs, int nwaves) {
    constexpr int R = Sh::R, H = Sh::H, DW = Sh::DW;
    auto rows = [](int q, int (&j)[4]) {
        int dA, dB;
        pair_rows<Sh>(q, dA, dB, j[0], j[1]);
        const int sgn = q / (DW / 4) == 0 ? 1 : -1;
        j[2] = dA / R == H - 1 ? j[0] + sgn * R : -1000;
        j[3] = dB / R == H - 1 ? j[1] + sgn * R : -1000;
    };
    int mine[4];
    rows(pw, mine);
    uint32_t pairs = 0;   // bit per row pair
    for (int q = 0; q < npairs; ++q) {
        int th[4];
        rows(q, th);
        bool near = q == pw;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 4; ++v) {
                const int d1 = mine[u] - th[v], d2 = th[u] - mine[v];
                near = near || (d1 >= -R && d1 <= R) || (d2 >= -R && d2 <= R);
            }
        if (near) pairs |= 1u << q;
    }
    uint32_t waves = 0;
    for (int w = 0; w < nwaves; ++w)
        if ((pairs >> (w % npairs)) & 1u) waves |= 1u << w;
    return waves;
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

template <class S, typename Real, int DW, int VX, int WX, int NF = 1>
struct MwdKernel {
    static constexpr int R = S::R;
    using Sh = DiamondShape<R, DW>;
    static constexpr int H = Sh::H, L = Sh::L;
    static constexpr int NPAIRS = DW / 2;       // waves along y (row pairs)
    static constexpr int NWAVES = NPAIRS * WX;  // WX waves along x per row pair
    static constexpr int NT = 64 * NWAVES;
    static_assert(NT <= 1024, "a workgroup holds at most 1024 threads");
    static constexpr int XL = 64 * VX * WX;     // x cells held per row
    static constexpr int XLP = XL + 2 * R;      // LDS sub-row stride (R guard cells per side)
    static constexpr int HX = R * (L - 1);      // redundant x halo per side
    static constexpr int XOWN_MAX = XL - 2 * HX;
    // Wavefront depth: a step advances NF planes (one "slab" of NF
    // consecutive planes per level); the z radius in slabs, and the skew of
    // the levels in slabs, is RZ = ceil(R / NF).
    static_assert(NF >= 1 && NF <= 4, "wavefront depth");
    // Box stencils read the level below at planes p-1, p, p+1 of the rows
    // beside their own: the levels are skewed by two planes (so that plane
    // p+1 is finished a step before it is read) and a stage row holds the
    // three planes, one sub-row each.  (Radius 1, one plane per step.)
    static constexpr bool BOX = S::BOX;
    static_assert(!BOX || (R == 1 && NF == 1), "box stencils: radius 1, one plane per step");
    static constexpr int RZ = BOX ? 2 : (R + NF - 1) / NF;
    // sub-rows of a stage row: the NF planes of a slab, or a box stencil's three
    static constexpr int SUB = BOX ? 3 : NF;
    // planes a duty stream (stage rows loaded from HBM) brings per step
    static constexpr int DP = BOX ? 3 : NF;
    static constexpr int SROW = SUB * XLP;
    // one stage buffer: stage rows plus 2R+1 spare rows that absorb the stage
    // writes and reads of slots without a stage row
    static constexpr int BUF_ROWS = Sh::STAGE_ROWS + 2 * R + 1;
    static constexpr int BUF_BYTES = BUF_ROWS * SROW * (int)sizeof(Real);
    // Two stage buffers (even and odd wavefront steps) when they fit in the
    // 160 KiB of LDS a workgroup may hold: a step then needs one barrier
    // (between staging and compute) instead of two.
    static constexpr bool DB = 2 * BUF_BYTES <= 163840;
    static constexpr int LDS_ROWS = BUF_ROWS * (DB ? 2 : 1);
    static constexpr int LDS_BYTES = LDS_ROWS * SROW * (int)sizeof(Real);
    static constexpr int RING = 2 * RZ;         // slabs a slot keeps along z
};

// Stage duties of one owned row.  Level k of the stage holds the time level
// t_c-H+k+1 that level k+1 reads.  A row's cells not computed in this diamond
// but read by its neighbours are the (at most two) levels just below its first
// computed level -- or, for a row the end of the run leaves empty, below the
// level it would have entered at -- and they come from the input pair.  A row
// that computes keeps level kf-1 in the slot of that level (its input ring),
// fed by one-step-ahead loads, and stages it like a computed level.
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

// Closed form of DiamondShape::srow0 for a level known only at run time.
template <class Sh>
__device__ __forceinline__ int srow0_rt(int k) {
    constexpr int R = Sh::R, H = Sh::H, DW = Sh::DW;
    const int base = k <= H ? R * k * (k + 3) : R * H * (H + 3) + (k - H) * DW - R * (k - H) * (k - H - 1);
    const int w1 = (k + 1) < H ? R * (k + 1) : DW / 2 - R * (k + 1 - H);
    return base - (DW / 2 - w1 - R);
}

// A wave-uniform value held in a vector register (keeps scalar registers free
// for what must be scalar).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t s) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// A wave-uniform value the compiler must treat as changed at this point, so
// that tests of its bits are made where they are used instead of being
// hoisted out of the wavefront loop as per-slot lane masks.
__device__ __forceinline__ uint32_t fresh_s(uint32_t x) {
    x = __builtin_amdgcn_readfirstlane(x);
    asm volatile("" : "+s"(x));
    return x;
}

// Same for a per-lane value: derived values are recomputed where used rather
// than precomputed per slot and kept alive (or spilled) across the loop.
__device__ __forceinline__ uint32_t fresh_v(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Buffer resource of a raw byte range starting at p (stride 0, 2^31 - 1
// bytes): stores whose offset is 2^31 or more fall outside the range and are
// dropped by the hardware's range check.
constexpr uint32_t DROP = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, 0x7fffffff, 0x00020000);
}
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rs, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, off, 0, 0);
}

// Bits lo..hi of a 32-bit mask (empty if lo > hi), clamped to 0..31.
__device__ __forceinline__ uint32_t bit_range(int lo, int hi) {
    lo = lo < 0 ? 0 : lo;
    hi = hi > 31 ? 31 : hi;
    return lo > hi ? 0u : (((2u << hi) - 1u) & ~((1u << lo) - 1u));
}

// Flag bits of a wave's scalar state.
enum : int {
    F_IN_A = 1 << 0, F_IN_B = 1 << 1,           // row inside the grid
    F_EDGE_X = 1 << 2, F_EDGE_Y = 1 << 3,       // workgroup touches the x / y halo
    F_CMP_A = 1 << 5, F_CMP_B = 1 << 6,         // row computes at least one level
    F_D1_A = 1 << 7, F_D2_A = 1 << 8, F_D1_B = 1 << 9, F_D2_B = 1 << 10,   // stage duties
    F_O_A = 1 << 11, F_O_B = 1 << 12,           // out-of-span duty
    F_PV_A = 1 << 13, F_PV_B = 1 << 14,         // parity of duty level kv's time level
    F_PT = 1 << 15,                             // parity of t_c
    F_COPY_A = 1 << 16, F_COPY_B = 1 << 17      // row inside the grid without a level in this row
};

// Every wave runs the same code: its two rows are laid out as one list of at
// most NS = L + 2 register slots -- row A's input level kfA-1 and its computed
// levels kfA..klA, then row B's input level and levels (a row that computes
// nothing keeps one unused slot).  A slot's level, LDS row and global offset
// are fixed per wave and precomputed; the ring of slot s (the last 2R planes
// of its level) lives in registers at a compile-time index.  Slots without a
// stage row of their own (unused slots, level L-1) write and read a block of
// spare LDS rows.  Where registers allow, the wavefront loop is unrolled over
// all 2R ring phases, so a ring advances by renaming its registers (always for
// R = 1); for larger R and wide or deep shapes the rings shift by one
// register per step instead, which keeps the loop free of spills.
//
// Two bodies share this state: the general one (any wavefront step) and the
// steady one, for steps at which the plane of every level lies inside the
// grid: it computes every slot without tests (unused slots compute values
// nobody reads) and keeps scalar work per step to a few tests.
//
// NSV (0 = L + 2) bounds the slot list: rows whose levels the start or the end
// of the run clips hold fewer slots per wave, and a kernel with fewer slots
// does proportionally less work per step.  The host launches such a kernel
// only for rows whose every wave fits (mwd_slots_needed).
//
// SY = 1: relaxed synchronisation (paper, Section "Multi-core wavefront
// temporal blocking": each thread waits only for the threads whose data it
// uses).  The two workgroup barriers of a step become waits on per-wave step
// counters in LDS: a wave stages step zs once the waves that read its stage
// rows have finished step zs-1 (zs-2 with two stage buffers), and updates
// once the waves whose rows it reads have staged step zs, so a wave that is
// ahead overlaps its staging with the update of waves that are behind.
// (Zero-halo instance only; the general-halo instance stages halo rows for
// other waves and keeps the barriers.)
template <class S, typename Real, int DW, int VX, int WX, int NSV, int NF, int SY = 0>
__device__ __forceinline__ void mwd_tile(const MwdArgs<Real>& a, const int64_t row_t_c, const int chunk,
                                         const int diamond, Real* __restrict__ stage,
                                         uint32_t* __restrict__ sync_flags = nullptr) {
    using KK = MwdKernel<S, Real, DW, VX, WX, NF>;
    using Sh = typename KK::Sh;
    constexpr int R = S::R, H = Sh::H, L = Sh::L, RING = KK::RING, XLP = KK::XLP, RZ = KK::RZ;
    constexpr int SROW = KK::SROW;
    constexpr int NS = NSV > 0 ? NSV : L + 2;
    static_assert(NS >= 3 && NS <= L + 2, "slot count");
    // steps unrolled per loop iteration, a multiple of the two stage buffers:
    // one per ring phase (2R) where that loop still compiles without spills
    // (at most four levels and 8 bytes per lane and ring plane), so the
    // z-rings rotate by renaming registers; otherwise two, and rings longer
    // than two planes shift by register moves
    constexpr int UNR = (RING == 2 || (L <= 4 && NF * VX * WX * (int)sizeof(Real) <= 8)) ? RING : 2;
    // HBM inputs are loaded PD steps before the step that uses them, into
    // one of PD register sets
    constexpr int PD = 1;
    // a slot's x/y neighbours are fetched LDEP slots ahead (from the stage;
    // x neighbours of FP64 radius-1 kernels from the neighbouring lanes)
    constexpr int LDEP = 1;
    // Rows that compute no level copy both input levels to the output pair.
    // Only the first and last diamond rows of a run hold such rows, and the
    // host runs those with the clipped-slot instance (NSV > 0), which has
    // registers to spare: there the copy is loaded one step ahead like every
    // other input.  The full instance, which meets such rows only when a
    // clipped row does not fit it, loads and stores in the same step.
    constexpr bool CPF = NSV > 0;
    constexpr int SB = (int)sizeof(Real);
    static_assert(NS <= 32, "slot masks are 32-bit");

    // ---- geometry (32-bit: sizes are bounded by the planner) ----------------
    const int nx = (int)a.g.nx, ny = (int)a.g.ny, nz = (int)a.g.nz, hh = a.g.h;
    const int pitchx = (int)a.g.pitch_x;
    const uint32_t plane_b = (uint32_t)(a.g.plane() * SB);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int pw = wave % KK::NPAIRS;              // row pair of this wave
    const int cb = 64 * VX * (wave / KK::NPAIRS);  // first column of this wave's x slice
    const int ybase = (int)(a.c_first + (int64_t)diamond * DW) - DW / 2;   // global y of local row 0
    const int x_own_lo = chunk * a.x_own;
    const int x_own_hi = x_own_lo + a.x_own < nx ? x_own_lo + a.x_own : nx;
    const int x0 = x_own_lo - KK::HX;              // x of column 0
    const int t_c = (int)row_t_c, T = (int)a.T;

    // per-lane constants: clamped byte offset within a row, ownership, x-halo
    uint32_t xb[VX], kill[VX];   // kill: DROP on lanes whose stores this chunk does not own
    bool xh[VX];
    // R = 1, FP64: x neighbours come from the neighbouring lanes' registers,
    // except at the ends of a 64-lane block and next to halo lanes (whose
    // registers hold no halo values), where they are read from the stage.
    // (FP32 kernels, two stage buffers, lose with it; radius 4 would need
    // eight moves per value.)
    constexpr bool XDPP = R == 1 && sizeof(Real) == 8 && !KK::BOX;
    bool mxm[VX], mxp[VX];
    auto in_halo = [&](int x) { return (x >= -R && x < 0) || (x >= nx && x < nx + R); };
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int x = x0 + cb + lane + 64 * v;
        const int xc = x < -R ? -R : (x >= nx + R ? nx + R - 1 : x);
        xb[v] = (uint32_t)((xc + hh) * SB);
        kill[v] = x >= x_own_lo && x < x_own_hi ? 0u : DROP;
        xh[v] = in_halo(x);
        mxm[v] = lane == 0 || in_halo(x - 1);
        mxp[v] = lane == 63 || in_halo(x + 1);
    }

    // ---- this wave's two rows ------------------------------------------------
    const int side = pw / (DW / 4);         // 0: right half (j >= DW/2), 1: left half
    int dA, dB, jA, jB;
    pair_rows<Sh>(pw, dA, dB, jA, jB);
    int kfA, klA, kfB, klB;
    row_levels<Sh>(jA, ybase + jA, ny, t_c, T, kfA, klA);
    row_levels<Sh>(jB, ybase + jB, ny, t_c, T, kfB, klB);
    auto in_layout = [&](int k, int j) -> bool {
        if (k < 0 || k > L - 2) return false;
        const int wk = (k + 1) < H ? R * (k + 1) : DW / 2 - R * (k + 1 - H);
        return j >= DW / 2 - wk - R && j < DW / 2 + wk + R;
    };
    // Stage duties of a row: levels kv (from the input ring when the row
    // computes, else from a prefetch register) and kv-1.
    auto duty_of = [&](int d, int j, int kf, int kl, int& kv, bool& d1, bool& d2) {
        kv = -1; d1 = d2 = false;
        const int y = ybase + j;
        if (y < 0 || y >= ny) return;
        const int kmax = T - 1 + H - t_c > L - 1 ? L - 1 : T - 1 + H - t_c;   // last level inside the run
        const int ks = d / R + 1;                      // level the diamond shape enters at
        kv = kf <= kl ? kf - 1 : (ks - 1 < kmax - 1 ? ks - 1 : kmax - 1);
        auto ok = [&](int k) { return k >= 0 && t_c - H + k + 1 >= 0 && in_layout(k, j); };
        d1 = kf > kl && ok(kv);
        d2 = ok(kv - 1);
    };
    int kvA, kvB;
    bool d1A, d2A, d1B, d2B;
    duty_of(dA, jA, kfA, klA, kvA, d1A, d2A);
    duty_of(dB, jB, kfB, klB, kvB, d1B, d2B);
    // The outermost block of rows reads, at level H, the rows up to R beyond
    // the diamond at level H-1 (time t_c).  The owner of an outermost row j
    // stages the row R further out (j+R on the right, j-R on the left); it does
    // so whether or not its own row is inside the grid.
    auto out_row = [&](int d, int j) -> int {
        if (d / R != H - 1 || t_c >= T) return -1000;
        const int jo = side == 0 ? j + R : j - R;
        const int yo = ybase + jo;
        return yo >= -R && yo < ny + R ? jo : -1000;
    };
    const int joA = out_row(dA, jA), joB = out_row(dB, jB);
    const bool inA = ybase + jA >= 0 && ybase + jA < ny, inB = ybase + jB >= 0 && ybase + jB < ny;
    const bool cmpA = kfA <= klA, cmpB = kfB <= klB;
    const bool edge_x = x0 < 0 || x0 + KK::XL > nx;           // chunk touches the x halo
    const bool edge_y = ybase - R < 0 || ybase + DW + R > ny;  // diamond touches the y halo
    const int zero_halo = __builtin_amdgcn_readfirstlane(*a.zero_halo);
    const int p0 = (t_c - H) & 1;   // parity of the time level of level 0
    const int flags = (inA ? F_IN_A : 0) | (inB ? F_IN_B : 0) | (edge_x ? F_EDGE_X : 0) |
                      (edge_y ? F_EDGE_Y : 0) | (cmpA ? F_CMP_A : 0) |
                      (cmpB ? F_CMP_B : 0) | (d1A ? F_D1_A : 0) | (d2A ? F_D2_A : 0) | (d1B ? F_D1_B : 0) |
                      (d2B ? F_D2_B : 0) | (joA > -1000 ? F_O_A : 0) | (joB > -1000 ? F_O_B : 0) |
                      (((t_c - H + kvA + 1) & 1) ? F_PV_A : 0) | (((t_c - H + kvB + 1) & 1) ? F_PV_B : 0) |
                      ((t_c & 1) ? F_PT : 0) | (inA && !cmpA ? F_COPY_A : 0) | (inB && !cmpB ? F_COPY_B : 0);
    auto rowb_of = [&](int j) -> uint32_t { return (uint32_t)((ybase + j + hh) * pitchx * SB); };
    // element index of (stage level k, local row j), sub-row 0 (sub-row f at + f*XLP)
    auto lds_row = [&](int k, int j) -> int { return (srow0_rt<Sh>(k) + j) * SROW + R; };
    const uint32_t lane_b = (uint32_t)((cb + lane) * SB);
    // LDS byte addresses (wave-uniform part; a lane adds lane_b) of the duty
    // rows, and byte offsets (uniform part; a lane adds its x offset) of the
    // prefetch streams from the base of their step's window (first plane of
    // slab zs + PD - RZ*L): a stream at depth dz reads slab zs + PD - RZ*dz of
    // its row (plane f of the slab at + f planes).
    // Kept uniform, so they cost scalar rather than vector registers.
    auto fo_of = [&](int dz, int j) -> uint32_t { return (uint32_t)(NF * RZ * (L - dz)) * plane_b + rowb_of(j); };
    const uint32_t uA2 = (uint32_t)(lds_row(kvA - 1, jA) * SB), uB2 = (uint32_t)(lds_row(kvB - 1, jB) * SB),
                   uOA = (uint32_t)(lds_row(H - 1, joA) * SB), uOB = (uint32_t)(lds_row(H - 1, joB) * SB);
    // second-order-in-time stencils: the first level kf of a computing row
    // also reads level kf-2 (time t-1) at its own cell, slab zs - RZ*kf
    const uint32_t foUA = fo_of(kvA + 1 < L ? kvA + 1 : 0, jA), foUB = fo_of(kvB + 1 < L ? kvB + 1 : 0, jB);
    const uint32_t foA = fo_of(kvA < 0 ? 0 : kvA, jA), foB = fo_of(kvB < 0 ? 0 : kvB, jB),
                   foOA = fo_of(H, joA > -1000 ? joA : jA), foOB = fo_of(H, joB > -1000 ? joB : jB);

    // ---- slot layout -----------------------------------------------------------
    const int sB = cmpA ? klA - kfA + 2 : 1;   // first slot of row B
    const int nB = cmpB ? klB - kfB + 2 : 1;
    // Level of each row's first slot: its input level kf-1 = kv.  A row that
    // computes nothing but owes level kv (d1) keeps it in that slot too: the
    // slot is loaded and staged exactly like an input ring.
    const int baseA = cmpA ? kfA - 1 : kvA, baseB = cmpB ? kfB - 1 : kvB;
    // LDS byte address (per lane) of the corner (row - R, column - R) of the
    // slot's stage row, and the slot's global byte offset within the step's
    // window (first plane of its level's slab, its row); masks over slots.
    constexpr int CORNER = (R * SROW + R) * SB;   // from the corner to the cell itself
    const uint32_t spare = (uint32_t)(Sh::STAGE_ROWS * SROW * SB);
    uint32_t lcs[NS], gos[S::NCOEF > 0 ? NS : 1];
    uint32_t cmS = 0;
    static_for<0, NS>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const bool isB = s >= sB;
        const int t = isB ? s - sB : s;
        const bool valid = isB ? (cmpB ? t < nB : (d1B && t == 0)) : (cmpA || d1A);
        const int k = (isB ? baseB : baseA) + t;
        const int j = isB ? jB : jA;
        lcs[s] = in_vgpr(valid ? (uint32_t)(lds_row(k, j) * SB - CORNER) : spare) + lane_b;
        if constexpr (S::NCOEF > 0) gos[s] = in_vgpr(valid ? (uint32_t)(NF * RZ * (L - k)) * plane_b + rowb_of(j) : 0u);
        cmS |= valid && t >= 1 ? 1u << s : 0u;
    });
    // Stores: the state a row leaves is its last two levels kl and kl-1 (for a
    // row with one level, kl-1 is its input level).  At step zs the stage row
    // of level k holds slab zs - RZ*(k+1), so the stores read the two stage
    // rows back after the barrier: every plane of each level passes through
    // the stage once.  Per row the even and the odd one of the two levels
    // (time levels of opposite parity) go to out[p0^1] and out[p0].
    // Store i: 0 = A even, 1 = A odd, 2 = B even, 3 = B odd (offsets of the
    // slab's first plane; plane f of the slab at + f planes).
    uint32_t stl[4], sgo[4][VX];
    int stk[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool isB = i >= 2;
        const bool cmp = isB ? cmpB : cmpA;
        const int kl = isB ? klB : klA;
        const int k = ((kl & 1) == (i & 1)) ? kl : kl - 1;   // level of this parity
        const int j = isB ? jB : jA;
        stk[i] = cmp ? k : -1000;
        stl[i] = in_vgpr(cmp ? (uint32_t)(lds_row(k, j) * SB) : spare) + lane_b;
        const uint32_t u = in_vgpr(cmp ? (uint32_t)(NF * RZ * (L - k - 1)) * plane_b + rowb_of(j) : 0u);
#pragma unroll
        for (int v = 0; v < VX; ++v) sgo[i][v] = cmp ? ((u + xb[v]) | kill[v]) : DROP;
    }
    // rows that compute no level copy both input levels: slab zs is RZ*L
    // slabs above the window base
    uint32_t cpo[2][VX];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint32_t u = in_vgpr((uint32_t)(NF * RZ * L) * plane_b + rowb_of(t == 0 ? jA : jB));
#pragma unroll
        for (int v = 0; v < VX; ++v) cpo[t][v] = u + xb[v];
    }
    const uint32_t maskA = bit_range(0, sB - 1);

    // Two instances of the sweep: zero Dirichlet halo (halo cells are
    // constants) and general halo (loaded where needed).
    auto sweep = [&](auto zhc) __attribute__((always_inline)) {
        constexpr bool ZH = decltype(zhc)::value;
        // relaxed synchronisation: per-wave counters of staged (sync_flags[w])
        // and updated (sync_flags[16 + w]) steps; step zs counts as zs + RING + 1
        constexpr bool RLX = SY != 0 && ZH;
        static_assert(SY == 0 || KK::NWAVES <= 16, "step counters for at most 16 waves");
        const uint32_t nbr = RLX ? pair_neighbours<Sh>(pw, KK::NPAIRS, KK::NWAVES) & ~(1u << wave) : 0u;
        bool gave_up = false;
        if constexpr (RLX) {
            if (threadIdx.x < 32) sync_flags[threadIdx.x] = 0u;
        }
        // counter of step zs in bank b (0: staged, 1: updated) of this wave
        auto post = [&](int b, int zs) __attribute__((always_inline)) {
            // the wave's LDS writes (b = 0) or reads (b = 1) of the step are
            // complete before the counter moves
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0)
                __hip_atomic_store(sync_flags + 16 * b + wave, (uint32_t)(zs + RING + 1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // wait until every neighbour's counter in bank b has reached step zs
        auto wait = [&](int b, int zs) __attribute__((always_inline)) {
            if (gave_up) return;
            const uint32_t want = (uint32_t)(zs + RING + 1);
            uint32_t spins = 0;
            for (;;) {
                // lane l reads wave l % 16's counter
                const uint32_t c = __hip_atomic_load(sync_flags + 16 * b + (lane & 15), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint64_t behind = __ballot((int32_t)(c - want) < 0) & (uint64_t)nbr;
                if (behind == 0) break;
                if (spins++ >= a.spin_limit) {
                    // cannot happen while every wave runs (each waits only on
                    // counters of earlier phases); bounded all the same
                    gave_up = true;
                    if (lane == 0) __hip_atomic_store(a.error, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                // (no sleep between polls: a wave waits a phase of a neighbour
                // at most, and a sleep would add its length to every wait)
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        };
        // Halo rows of the stage (rows outside the grid, inside it +-R): with a zero
        // halo they are written once here and never touched again.
        if (ZH && edge_y) {
            for (int k = 0; k < L - 1; ++k) {
                for (int j = Sh::sl_lo(k); j < Sh::sl_lo(k) + Sh::nrows(k); ++j) {
                    const int y = ybase + j;
                    if ((y >= -R && y < 0) || (y >= ny && y < ny + R)) {
                        for (int b = 0; b < (KK::DB ? 2 : 1); ++b) {
                            Real* sp = stage + b * KK::BUF_ROWS * SROW + lds_row(k, j) - R;
                            for (int col = threadIdx.x; col < SROW; col += KK::NT) sp[col] = Real(0);
                        }
                    }
                }
            }
        }
        // Zero halo, workgroups at the x edge: the x-halo lanes zero their
        // column of every stage row once and never stage anything (their
        // writes are masked off), so interior workgroups stage without
        // selects or extra writes.
        bool hz[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) hz[v] = ZH && edge_x && xh[v];
        if (ZH && edge_x) {
#pragma unroll
            for (int v = 0; v < VX; ++v)
                if (hz[v])
                    for (int row = 0; row < KK::LDS_ROWS * KK::SUB; ++row) stage[row * XLP + R + cb + lane + 64 * v] = Real(0);
        }

        // wavefront steps end here: the last slab of level L-1 (slab nzq-1) is
        // computed at step nzq-1 + RZ*(L-1) and passes through the stage RZ
        // steps later
        const int nzq = (nz + NF - 1) / NF;
        const int nzs = nzq + RZ * L;
        // byte offset of plane q from the array base
        auto plane_off = [&](int q) -> int64_t { return (int64_t)(q + hh) * (int64_t)plane_b; };
        auto at = [](const Real* base, int64_t off) -> const Real* {
            return reinterpret_cast<const Real*>(reinterpret_cast<const char*>(base) + off);
        };
        auto atw = [](Real* base, int64_t off) -> Real* {
            return reinterpret_cast<Real*>(reinterpret_cast<char*>(base) + off);
        };
        auto lds = [&](uint32_t byte_addr) -> Real& {
            return *reinterpret_cast<Real*>(reinterpret_cast<char*>(stage) + byte_addr);
        };
        constexpr int DP = KK::DP;
        auto put = [&](uint32_t la, const Real (&src)[DP][VX]) {   // la: per-lane LDS byte address
#pragma unroll
            for (int f = 0; f < DP; ++f)
#pragma unroll
                for (int v = 0; v < VX; ++v)
                    if (!hz[v]) lds(la + (f * XLP + 64 * v) * SB) = src[f][v];
        };
        // x-halo columns of a staged computed row (slab q; a box stencil's
        // planes q-1 .. q+1) when the halo is not zero
        auto fix_halo_cols = [&](int li, int q, int y) {   // li: element index, buffer included
#pragma unroll
            for (int f = 0; f < KK::SUB; ++f) {
                const int pl = KK::BOX ? q - 1 + f : NF * q + f;
                if (pl < -R || pl >= nz + R) continue;
                const Real* base = at(a.in[0], plane_off(pl) + (int64_t)(y + hh) * pitchx * SB);
#pragma unroll
                for (int v = 0; v < VX; ++v)
                    if (xh[v]) stage[li + f * XLP + cb + lane + 64 * v] = ld_at(base, xb[v]);
            }
        };

        // Loads of step zs + PD's inputs (see the streams above); with a
        // staging function, duty registers are first staged.
        auto prefetch = [&](int zs, bool steady, Real (&vA)[NF][VX], Real (&vB)[NF][VX], Real (&dA2)[DP][VX],
                            Real (&dB2)[DP][VX], Real (&rA)[DP][VX], Real (&rB)[DP][VX], Real (&wA)[NF][VX],
                            Real (&wB)[NF][VX], auto&& stage_fn) __attribute__((always_inline)) {
            const int f = (int)fresh_s((uint32_t)flags);
            // per-lane offsets, formed here from the uniform parts (fresh
            // copies keep the compiler from hoisting them into registers
            // that stay live across the loop)
            uint32_t oA[VX], oB[VX], oOA[VX], oOB[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                oA[v] = fresh_s(foA) + xb[v];
                oB[v] = fresh_s(foB) + xb[v];
                oOA[v] = fresh_s(foOA) + xb[v];
                oOB[v] = fresh_s(foOB) + xb[v];
            }
            const int64_t nb = plane_off(NF * (zs + PD - RZ * L));
            const Real* fb0 = at(a.in[0], nb);
            const Real* fb1 = at(a.in[1], nb);
            auto fetch = [&](bool odd, int dz, const uint32_t (&o)[VX], Real (&dst)[NF][VX]) __attribute__((always_inline)) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if (!steady) {
                        const int q = NF * (zs + PD - RZ * dz) + f;
                        if (q < -R || q >= nz + R) continue;
                    }
                    const Real* base = at(odd ? fb1 : fb0, (int64_t)f * plane_b);
#pragma unroll
                    for (int v = 0; v < VX; ++v) dst[f][v] = ld_at(base, o[v]);
                }
            };
            // duty streams: the NF planes of the slab, or a box stencil's
            // planes p-1 .. p+1 around its plane p (inside the haloed grid in
            // the steady range: p+1 is at least one slab below zs + PD)
            auto fetchd = [&](bool odd, int dz, const uint32_t (&o)[VX], Real (&dst)[DP][VX]) __attribute__((always_inline)) {
#pragma unroll
                for (int f = 0; f < DP; ++f) {
                    const int df = KK::BOX ? f - 1 : f;
                    if (!steady) {
                        const int q = NF * (zs + PD - RZ * dz) + df;
                        if (q < -R || q >= nz + R) continue;
                    }
                    const Real* base = at(odd ? fb1 : fb0, (int64_t)df * plane_b);
#pragma unroll
                    for (int v = 0; v < VX; ++v) dst[f][v] = ld_at(base, o[v]);
                }
            };
            if (f & (F_CMP_A | F_D1_A)) fetch(f & F_PV_A, kvA, oA, vA);
            if (f & (F_CMP_B | F_D1_B)) fetch(f & F_PV_B, kvB, oB, vB);
            if (f & F_D2_A) { stage_fn(fresh_s(uA2) + lane_b, dA2); fetchd(!(f & F_PV_A), kvA, oA, dA2); }
            if (f & F_D2_B) { stage_fn(fresh_s(uB2) + lane_b, dB2); fetchd(!(f & F_PV_B), kvB, oB, dB2); }
            if (f & F_O_A) { stage_fn(fresh_s(uOA) + lane_b, rA); fetchd(f & F_PT, H, oOA, rA); }
            if (f & F_O_B) { stage_fn(fresh_s(uOB) + lane_b, rB); fetchd(f & F_PT, H, oOB, rB); }
            if constexpr (S::LEAPFROG) {
                // level kf-2 of a computing row: the time level of parity
                // opposite to kv's, slab zs + PD - RZ*kf
                uint32_t oU[VX];
                if (f & F_CMP_A) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) oU[v] = fresh_s(foUA) + xb[v];
                    fetch(!(f & F_PV_A), kvA + 1, oU, wA);
                }
                if (f & F_CMP_B) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) oU[v] = fresh_s(foUB) + xb[v];
                    fetch(!(f & F_PV_B), kvB + 1, oU, wB);
                }
            }
        };

        Real ring[NS][RING][NF][VX];
        // Prefetch registers, one set per step parity.  qA/qB: the input level
        // kv of a row (its input ring);
        // p2: duty level kv-1; po: the out-of-span row.
        Real qA[PD][NF][VX], qB[PD][NF][VX], p2A[PD][DP][VX], p2B[PD][DP][VX], poA[PD][DP][VX], poB[PD][DP][VX];
        // second-order-in-time stencils: level kf-2 of each row (the first
        // computed level's previous time level)
        Real uA[PD][NF][VX], uB[PD][NF][VX];
        // copied levels (row A / B, input array 0 / 1) of slab zs + PD
        Real cpv[PD][2][2][NF][VX];
#pragma unroll
        for (int f = 0; f < DP; ++f)
#pragma unroll
            for (int v = 0; v < VX; ++v)
#pragma unroll
                for (int c = 0; c < PD; ++c) p2A[c][f][v] = p2B[c][f][v] = poA[c][f][v] = poB[c][f][v] = Real(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
#pragma unroll
                for (int c = 0; c < PD; ++c) {
                    qA[c][f][v] = qB[c][f][v] = Real(0);
                    uA[c][f][v] = uB[c][f][v] = Real(0);
                    cpv[c][0][0][f][v] = cpv[c][0][1][f][v] = cpv[c][1][0][f][v] = cpv[c][1][1][f][v] = Real(0);
                }
#pragma unroll
                for (int m = 0; m < RING; ++m) {
#pragma unroll
                    for (int i = 0; i < NS; ++i) ring[i][m][f][v] = Real(0);
                }
            }
        }

        // One wavefront step; ph: step index modulo UNR.
        auto step = [&](auto phc, auto steadyc, int zs, auto sbc) __attribute__((always_inline)) {
            // row B's first slot: a compile-time index where the caller knows it (SBK >= 0)
            constexpr int SBK = decltype(sbc)::value;
            constexpr int ph = decltype(phc)::value;
            constexpr bool STEADY = decltype(steadyc)::value;
            // stage buffer of this step (steps start at an even zs, so ph = zs mod 2)
            constexpr uint32_t BOFF = KK::DB ? (uint32_t)(ph & 1) * KK::BUF_BYTES : 0u;
            constexpr int BOFE = (int)BOFF / SB;
            // physical register of logical ring position m (0 = oldest plane)
            auto P = [](int m) { return UNR == RING ? (m + ph) % RING : m; };
            const bool live = STEADY || UNR == 1 || zs < nzs;   // uniform across the workgroup
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                lcs[i] = fresh_v(lcs[i]);
                gos[i] = fresh_v(gos[i]);
            }
            Real vcA[NF][VX], vcB[NF][VX], vuA[NF][VX], vuB[NF][VX];
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    vcA[f][v] = qA[ph % PD][f][v];
                    vcB[f][v] = qB[ph % PD][f][v];
                    vuA[f][v] = uA[ph % PD][f][v];
                    vuB[f][v] = uB[ph % PD][f][v];
                }
            // the readers of this wave's stage rows are done with the buffer
            if constexpr (RLX) wait(1, zs - (KK::DB ? 2 : 1));
            // ---- A: stage every plane the levels read this step ------------------
            if (live) {
                const int f = (int)fresh_s((uint32_t)flags);
                // copied levels of slab zs, loaded one step ago (before this
                // step's loads reuse the registers)
                if constexpr (CPF) {
                    if ((f & (F_COPY_A | F_COPY_B)) && zs >= 0 && NF * zs < nz) {
                        const int64_t e0b = plane_off(NF * (zs - RZ * L));
                        const __amdgpu_buffer_rsrc_t o0 = raw_rsrc(atw(a.out[0], e0b)),
                                                     o1 = raw_rsrc(atw(a.out[1], e0b));
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            if (f & (t == 0 ? F_COPY_A : F_COPY_B)) {
#pragma unroll
                                for (int g = 0; g < NF; ++g) {
                                    // planes of the slab beyond the grid are dropped
                                    const uint32_t zd = NF * zs + g < nz ? 0u : DROP;
#pragma unroll
                                    for (int v = 0; v < VX; ++v) {
                                        const uint32_t o = (cpo[t][v] + g * plane_b) | kill[v] | zd;
                                        buf_store(o0, o, cpv[ph % PD][t][0][g][v]);
                                        buf_store(o1, o, cpv[ph % PD][t][1][g][v]);
                                    }
                                }
                            }
                        }
                    }
                }
                // every slot (unused ones into the spare rows); the duty rows are
                // written after them
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    if (!hz[v]) {
                        static_for<0, NS>([&](auto sc) __attribute__((always_inline)) {
                            constexpr int s = decltype(sc)::value;
                            if constexpr (KK::BOX) {
                                // planes p-1, p, p+1 of the level: ring positions RZ-1 .. RZ+1
#pragma unroll
                                for (int d = 0; d < 3; ++d)
                                    lds(lcs[s] + BOFF + CORNER + (d * XLP + 64 * v) * SB) = ring[s][P(RZ - 1 + d)][0][v];
                            } else {
#pragma unroll
                                for (int g = 0; g < NF; ++g)
                                    lds(lcs[s] + BOFF + CORNER + (g * XLP + 64 * v) * SB) = ring[s][P(RZ)][g][v];
                            }
                        });
                    }
                }
                // loads for step zs + PD into this step's register set (its
                // values are consumed above or copied to vcA/vcB): slab
                // zs + PD - RZ*dz of each stream; planes outside the haloed grid
                // are skipped (no computing cell reads them; in the steady range
                // every plane is inside).  A duty register is staged before its
                // next load is issued.
                prefetch(zs, STEADY, qA[ph % PD], qB[ph % PD], p2A[ph % PD], p2B[ph % PD], poA[ph % PD], poB[ph % PD],
                         uA[ph % PD], uB[ph % PD],
                         [&](uint32_t la, const Real (&src)[DP][VX]) __attribute__((always_inline)) { put(la + BOFF, src); });
                if constexpr (CPF) {
                    const int q = zs + PD;   // the slab the copy stores at step zs + PD
                    if ((f & (F_COPY_A | F_COPY_B)) && q >= 0 && NF * q < nz) {
                        const int64_t nb = plane_off(NF * (q - RZ * L));
#pragma unroll
                        for (int g = 0; g < NF; ++g) {
                            if (NF * q + g >= nz) continue;
                            const Real* fb0 = at(a.in[0], nb + (int64_t)g * plane_b);
                            const Real* fb1 = at(a.in[1], nb + (int64_t)g * plane_b);
#pragma unroll
                            for (int t = 0; t < 2; ++t) {
                                if (f & (t == 0 ? F_COPY_A : F_COPY_B)) {
#pragma unroll
                                    for (int v = 0; v < VX; ++v) {
                                        cpv[ph % PD][t][0][g][v] = ld_at(fb0, cpo[t][v]);
                                        cpv[ph % PD][t][1][g][v] = ld_at(fb1, cpo[t][v]);
                                    }
                                }
                            }
                        }
                    }
                }
                // non-zero halo, edge workgroups only: fixed values in halo columns
                // of computed rows, and halo rows (latency exposed)
                if (!ZH && (f & (F_EDGE_X | F_EDGE_Y))) {
                    if (f & F_EDGE_X) {
                        for (int k = kfA; k <= klA && k <= L - 2; ++k)
                            fix_halo_cols(lds_row(k, jA) + BOFE, zs - RZ * (k + 1), ybase + jA);
                        for (int k = kfB; k <= klB && k <= L - 2; ++k)
                            fix_halo_cols(lds_row(k, jB) + BOFE, zs - RZ * (k + 1), ybase + jB);
                    }
                    if (f & F_EDGE_Y) {
                        for (int k = wave; k < L - 1; k += KK::NWAVES) {
                            for (int j = Sh::sl_lo(k); j < Sh::sl_lo(k) + Sh::nrows(k); ++j) {
                                const int y = ybase + j;
                                if (!((y >= -R && y < 0) || (y >= ny && y < ny + R))) continue;
                                for (int g = 0; g < KK::SUB; ++g) {
                                    const int q = KK::BOX ? zs - RZ * (k + 1) - 1 + g : NF * (zs - RZ * (k + 1)) + g;
                                    if (q < -R || q >= nz + R) continue;
                                    const Real* base = at(a.in[0], plane_off(q) + (int64_t)(y + hh) * pitchx * SB);
                                    const int li = lds_row(k, j) + BOFE + g * XLP;
                                    for (int col = lane; col < KK::XL; col += 64) {
                                        const int x = x0 + col;
                                        const int xc = x < -R ? -R : (x >= nx + R ? nx + R - 1 : x);
                                        stage[li + col] = base[xc + hh];
                                    }
                                }
                            }
                        }
                    }
                }
            }
            if constexpr (RLX) {
                post(0, zs);
                wait(0, zs);
            } else {
                __syncthreads();
            }
            // ---- B: update every (row, level) slot of this step ----------------------
            if (live) {
                const int f = (int)fresh_s((uint32_t)flags);
                // window of this step: slabs [zs - RZ*L, zs]
                const int64_t e0b = plane_off(NF * (zs - RZ * L));
                // the rows' last two levels, from the stage (see above).  With
                // one stage buffer they are read back after the update, when
                // waves that finished early would otherwise wait at the
                // barrier; with two, before it (there is no such wait to fill).
                auto store_levels = [&]() __attribute__((always_inline)) {
                    const __amdgpu_buffer_rsrc_t rs_even = raw_rsrc(atw(a.out[p0 ^ 1], e0b));
                    const __amdgpu_buffer_rsrc_t rs_odd = raw_rsrc(atw(a.out[p0], e0b));
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
#pragma unroll
                        for (int g = 0; g < NF; ++g) {
                            uint32_t zd = 0;
                            if constexpr (!STEADY) {
                                const int q = NF * (zs - RZ * (stk[i] + 1)) + g;
                                zd = q >= 0 && q < nz ? 0u : DROP;
                            }
#pragma unroll
                            for (int v = 0; v < VX; ++v)
                                buf_store((i & 1) ? rs_odd : rs_even, (sgo[i][v] + g * plane_b) | zd,
                                          lds(stl[i] + BOFF + ((KK::BOX ? 1 : g) * XLP + 64 * v) * SB));
                        }
                    }
                };
                if constexpr (KK::DB) store_levels();
                const uint32_t cm = fresh_s(cmS);
                const int sb = (int)fresh_s((uint32_t)sB);
                // per plane g of the slab: slots whose level's plane
                // NF*(zs - RZ*k) + g lies inside the grid
                uint32_t zS[NF];
#pragma unroll
                for (int g = 0; g < NF; ++g) {
                    zS[g] = 0xffffffffu;
                    if constexpr (!STEADY) {
                        const int pz = NF * zs + g;
                        const int khz = pz >= 0 ? pz / (NF * RZ) : -1;
                        const int klz = pz - nz >= 0 ? (pz - nz) / (NF * RZ) + 1 : 0;
                        zS[g] = (bit_range(klz - baseA, khz - baseA) & maskA) |
                                (bit_range(klz - baseB + sB, khz - baseB + sB) & ~maskA);
                    }
                }
                Real prev[NF][VX];
                // second-order-in-time stencils: level k-2 at a slot's own cell,
                // the oldest slab of the ring two slots back, taken from it
                // before the previous slot's iteration overwrites it
                Real uold[NF][VX];
                // x/y neighbours of a slot, read from the stage one slot ahead
                // of its use (a one-deep software pipeline: deeper prefetching
                // would hold too many registers)
                Real nb[LDEP + 1][4 * R][NF][VX];
                // coefficients of a slot's plane (stencils with coefficient
                // arrays), loaded with its neighbours, LDEP slots ahead: in the
                // steady range every slot's offset (0 for unused slots: the
                // window's first plane, NF*(zs - RZ*L) >= 0) stays inside the
                // arrays; elsewhere only slots whose plane is inside the grid load
                Real cfp[LDEP + 1][S::NCOEF > 0 ? S::NCOEF : 1][NF][VX];
                auto load_nb = [&](auto tc) __attribute__((always_inline)) {
                    constexpr int t = decltype(tc)::value;
                    if constexpr (S::NCOEF > 0) {
#pragma unroll
                        for (int g = 0; g < NF; ++g) {
                            const bool zvt = ((cm & zS[g]) >> t) & 1u;
#pragma unroll
                            for (int v = 0; v < VX; ++v) {
                                if (STEADY || zvt) {
                                    const uint32_t go = gos[t] + xb[v];
#pragma unroll
                                    for (int m = 0; m < S::NCOEF; ++m)
                                        cfp[t % (LDEP + 1)][m][g][v] =
                                            ld_at(at(a.coef.arr[m], e0b + (int64_t)g * plane_b), go);
                                } else {
#pragma unroll
                                    for (int m = 0; m < S::NCOEF; ++m) cfp[t % (LDEP + 1)][m][g][v] = Real(0);
                                }
                            }
                        }
                    }
                    // (box stencils read their neighbourhood in the slot itself)
                    const uint32_t lb = lcs[t - 1] + BOFF;     // corner of (level - 1, row)
#pragma unroll
                    for (int g = 0; g < (KK::BOX ? 0 : NF); ++g) {
#pragma unroll
                        for (int v = 0; v < VX; ++v) {
                            const uint32_t c0 = lb + (g * XLP + 64 * v) * SB + CORNER;
                            if constexpr (XDPP) {
                                // the level below's plane at the neighbouring lanes is
                                // what they staged: their ring position RZ
                                nb[t % (LDEP + 1)][2][g][v] = lds(c0 + SROW * SB);
                                nb[t % (LDEP + 1)][3][g][v] = lds(c0 - SROW * SB);
                                const Real cc = ring[t - 1][P(RZ)][g][v];
                                Real xp = lane_shift<0x130>(cc), xm = lane_shift<0x138>(cc);
                                if (mxp[v]) xp = lds(c0 + SB);
                                if (mxm[v]) xm = lds(c0 - SB);
                                nb[t % (LDEP + 1)][0][g][v] = xp;
                                nb[t % (LDEP + 1)][1][g][v] = xm;
                            } else {
#pragma unroll
                                for (int r = 1; r <= R; ++r) {
                                    nb[t % (LDEP + 1)][r - 1][g][v] = lds(c0 + r * SB);
                                    nb[t % (LDEP + 1)][R + r - 1][g][v] = lds(c0 - r * SB);
                                    nb[t % (LDEP + 1)][2 * R + r - 1][g][v] = lds(c0 + r * SROW * SB);
                                    nb[t % (LDEP + 1)][3 * R + r - 1][g][v] = lds(c0 - r * SROW * SB);
                                }
                            }
                        }
                    }
                };
                static_for<1, (LDEP + 1 < NS ? LDEP + 1 : NS)>([&](auto tc) __attribute__((always_inline)) { load_nb(tc); });
                static_for<0, NS>([&](auto sc) __attribute__((always_inline)) {
                    constexpr int s = decltype(sc)::value;
                    // Wave priority falls as a wave advances through its slots,
                    // so a wave that is behind issues first.  (With equal
                    // priorities the oldest wave on a SIMD issues first, finishes
                    // first and waits at the barrier for the youngest, which runs
                    // its last slots alone.)
                    constexpr int PRI = 3 - (4 * s) / NS;
                    if constexpr (s == 0 || PRI != 3 - (4 * (s - 1)) / NS) __builtin_amdgcn_s_setprio(PRI);
                    Real nv[NF][VX];
                    if constexpr (s == 0) {
#pragma unroll
                        for (int g = 0; g < NF; ++g)
#pragma unroll
                            for (int v = 0; v < VX; ++v) nv[g][v] = vcA[g][v];
                    } else {
                        // every slot is computed (unused slots compute values nobody reads)
                        if constexpr (s + LDEP < NS) load_nb(std::integral_constant<int, s + LDEP>{});
                        // issue those reads before this slot's arithmetic
                        __builtin_amdgcn_sched_barrier(0);
                        if constexpr (SBK >= 0 && s == SBK) {
                            // row B's input slot takes the loaded input slab (no arithmetic)
#pragma unroll
                            for (int g = 0; g < NF; ++g)
#pragma unroll
                                for (int v = 0; v < VX; ++v) nv[g][v] = vcB[g][v];
                        } else {
#pragma unroll
                            for (int g = 0; g < NF; ++g) {
                                // a computed level whose plane g lies inside the grid
                                // (unused slots never count: their offsets are not
                                // theirs to load)
                                const bool zv = ((cm & zS[g]) >> s) & 1u;
#pragma unroll
                                for (int v = 0; v < VX; ++v) {
                                    if constexpr (KK::BOX) {
                                        // the 3x3x3 box of level k-1: the own column from the
                                        // ring (planes p-1, p, p+1 at positions RZ-1 .. RZ+1),
                                        // the rest from the stage (sub-row dz+1 holds plane p+dz)
                                        Box27<Real> bx;
                                        const uint32_t c0 = lcs[s - 1] + BOFF + 64 * v * SB + CORNER;
#pragma unroll
                                        for (int m = 0; m < 27; ++m) {
                                            const int dz = m / 9 - 1, dy = (m / 3) % 3 - 1, dx = m % 3 - 1;
                                            if (dy == 0 && dx == 0)
                                                bx.v[m] = ring[s - 1][P(RZ + dz)][0][v];
                                            else
                                                bx.v[m] = lds(c0 + ((dz + 1) * XLP + dy * SROW + dx) * SB);
                                        }
                                        nv[g][v] = Stencil27B::apply_box(bx, a.coef.k);
                                    } else {
                                        Nbhd<Real, R> n;
                                        n.c = ring[s - 1][P(RZ)][g][v];
                                        if constexpr (S::LEAPFROG) {
                                            // the first computed level of a row takes
                                            // level kf-2 from its HBM stream
                                            if constexpr (s == 1)
                                                n.uo = vuA[g][v];
                                            else if constexpr (SBK >= 0)
                                                n.uo = s == SBK + 1 ? vuB[g][v] : uold[g][v];
                                            else
                                                n.uo = s == sb + 1 ? vuB[g][v] : uold[g][v];
                                        }
#pragma unroll
                                        for (int r = 1; r <= R; ++r) {
                                            // plane g -/+ r of the slab: slab offset floor((g -/+ r) / NF),
                                            // plane within it; ring position RZ + that offset, where
                                            // position 2*RZ is the slab slot s-1 computed this step
                                            const int dm = g - r, dp = g + r;
                                            const int sm = dm >= 0 ? dm / NF : -((-dm + NF - 1) / NF);
                                            const int sp = dp / NF;
                                            n.zm[r - 1] = ring[s - 1][P(RZ + sm)][dm - sm * NF][v];
                                            n.zp[r - 1] = RZ + sp == RING ? prev[dp - sp * NF][v]
                                                                          : ring[s - 1][P(RZ + sp)][dp - sp * NF][v];
                                            n.xp[r - 1] = nb[s % (LDEP + 1)][r - 1][g][v];
                                            n.xm[r - 1] = nb[s % (LDEP + 1)][R + r - 1][g][v];
                                            n.yp[r - 1] = nb[s % (LDEP + 1)][2 * R + r - 1][g][v];
                                            n.ym[r - 1] = nb[s % (LDEP + 1)][3 * R + r - 1][g][v];
                                        }
                                        Real cf[S::NCOEF > 0 ? S::NCOEF : 1];
                                        if constexpr (S::NCOEF > 0) {
#pragma unroll
                                            for (int m = 0; m < S::NCOEF; ++m) cf[m] = cfp[s % (LDEP + 1)][m][g][v];
                                        }
                                        nv[g][v] = S::apply(n, a.coef.k, cf);
                                    }
                                }
                                if constexpr (!STEADY) {
                                    // a level whose plane is a halo plane (or beyond) holds the halo
                                    if (!zv) {
#pragma unroll
                                        for (int v = 0; v < VX; ++v) nv[g][v] = Real(0);
                                        if constexpr (!ZH) {
                                            // halo values, for computed levels only (an unused
                                            // slot's row may lie outside the grid)
                                            const bool isB = s >= sb;
                                            const int k = isB ? baseB + (s - sb) : baseA + s;
                                            const int q = NF * (zs - RZ * k) + g;
                                            if (((cm >> s) & 1u) && q >= -R && q < nz + R) {
                                                const Real* base = at(
                                                    a.in[0], plane_off(q) + (int64_t)(ybase + (isB ? jB : jA) + hh) * pitchx * SB);
#pragma unroll
                                                for (int v = 0; v < VX; ++v) nv[g][v] = ld_at(base, xb[v]);
                                            }
                                        }
                                    }
                                }
                            }
                            // row B's input slot takes the loaded input slab
                            if constexpr (SBK < 0) {
                                if (s == sb) {
#pragma unroll
                                    for (int g = 0; g < NF; ++g)
#pragma unroll
                                        for (int v = 0; v < VX; ++v) nv[g][v] = vcB[g][v];
                                }
                            }
                        }
                        // slot s-1's ring takes its newest slab (its oldest, level
                        // k-2 of slot s+1, kept first)
#pragma unroll
                        for (int g = 0; g < NF; ++g) {
#pragma unroll
                            for (int v = 0; v < VX; ++v) {
                                if constexpr (S::LEAPFROG) uold[g][v] = UNR == RING ? ring[s - 1][P(0)][g][v]
                                                                                     : ring[s - 1][0][g][v];
                                if constexpr (UNR == RING) {
                                    ring[s - 1][P(0)][g][v] = prev[g][v];
                                } else {
#pragma unroll
                                    for (int m = 0; m + 1 < RING; ++m) ring[s - 1][m][g][v] = ring[s - 1][m + 1][g][v];
                                    ring[s - 1][RING - 1][g][v] = prev[g][v];
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int g = 0; g < NF; ++g) {
#pragma unroll
                        for (int v = 0; v < VX; ++v) {
                            // pin the slot's result here: the arithmetic of a slot
                            // must not sink below later slots' reads, whose results
                            // would otherwise all be held in registers at once
                            asm volatile("" : "+v"(nv[g][v]));
                            prev[g][v] = nv[g][v];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                });
#pragma unroll
                for (int g = 0; g < NF; ++g) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        if constexpr (UNR == RING) {
                            ring[NS - 1][P(0)][g][v] = prev[g][v];
                        } else {
#pragma unroll
                            for (int m = 0; m + 1 < RING; ++m) ring[NS - 1][m][g][v] = ring[NS - 1][m + 1][g][v];
                            ring[NS - 1][RING - 1][g][v] = prev[g][v];
                        }
                    }
                }
                if constexpr (!KK::DB) store_levels();
                // rows of this diamond with no level in this row: carry both
                // levels (the clipped instance stored them in phase A)
                if (!CPF && (f & (F_COPY_A | F_COPY_B)) && zs >= 0 && NF * zs < nz) {
                    const __amdgpu_buffer_rsrc_t o0 = raw_rsrc(atw(a.out[0], e0b)), o1 = raw_rsrc(atw(a.out[1], e0b));
#pragma unroll
                    for (int g = 0; g < NF; ++g) {
                        if (NF * zs + g >= nz) continue;
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            if (f & (t == 0 ? F_COPY_A : F_COPY_B)) {
#pragma unroll
                                for (int v = 0; v < VX; ++v) {
                                    const uint32_t o = cpo[t][v] + g * plane_b;
                                    buf_store(o0, o | kill[v], ld_at(at(a.in[0], e0b), o));
                                    buf_store(o1, o | kill[v], ld_at(at(a.in[1], e0b), o));
                                }
                            }
                        }
                    }
                }
            }
            if constexpr (RLX)
                post(1, zs);
            else if constexpr (!KK::DB)
                __syncthreads();   // with two buffers the next step's staging may overlap
        };

        // the sweep starts 2*RZ steps early so that the input rings of rows
        // entering at level 1 hold the halo planes -R..-1; steps [zA, zB) are
        // steady: every plane of every level's slab zs - RZ*k (k = 0..L-1) and
        // of every stored slab zs - RZ*(k+1) is inside the grid
        const int zA = ((RZ * L + UNR - 1) / UNR) * UNR;
        // (slab zs's planes end at or below nz, and the planes of slab zs + PD,
        // loaded one step ahead, stay inside the haloed grid)
        const int zB1 = nz / NF, zB2 = (nz + R - NF) / NF - PD + 1;
        const int zB0 = zB1 < zB2 ? zB1 : zB2;
        const int zB = (zB0 / UNR) * UNR > zA ? (zB0 / UNR) * UNR : zA;
        // first loads: the inputs of steps -RING and -RING + 1
        auto no_stage = [](uint32_t, const Real (&)[DP][VX]) {};
        static_for<0, PD>([&](auto pc) __attribute__((always_inline)) {
            constexpr int c = decltype(pc)::value;
            prefetch(-RING - PD + c, false, qA[c], qB[c], p2A[c], p2B[c], poA[c], poB[c], uA[c], uB[c], no_stage);
        });
        __syncthreads();
        using General = std::integral_constant<bool, false>;
        using Steady = std::integral_constant<bool, true>;
        // (three loops rather than one with a per-step branch: separate loops
        // keep the register assignment of both bodies spill-free)
        using AnySB = std::integral_constant<int, -1>;
        int zb = -RING;
        for (; zb < nzs; zb += UNR) {
            if (zb >= zA && zb < zB) break;
            static_for<0, UNR>([&](auto phc) __attribute__((always_inline)) {
                step(phc, General{}, zb + decltype(phc)::value, AnySB{});
            });
        }
        // The steady loop is compiled once per position of row B's first slot
        // that a full diamond row has (L - 2b for b = 0 .. H/2 - 1), so that
        // slot skips the arithmetic and no slot selects at run time; other
        // positions (clipped rows) take the generic copy.
        auto steady = [&](auto sbc) __attribute__((always_inline)) {
            for (; zb < zB; zb += UNR)
                static_for<0, UNR>([&](auto phc) __attribute__((always_inline)) {
                    step(phc, Steady{}, zb + decltype(phc)::value, sbc);
                });
        };
        bool done = false;
        static_for<0, (H / 2 > 0 ? H / 2 : 1)>([&](auto bc) __attribute__((always_inline)) {
            constexpr int K = L - 2 * decltype(bc)::value;
            if (!done && K < NS && sB == K) {
                steady(std::integral_constant<int, (K < NS ? K : -1)>{});
                done = true;
            }
        });
        if (!done) steady(AnySB{});
        for (; zb < nzs; zb += UNR)
            static_for<0, UNR>([&](auto phc) __attribute__((always_inline)) {
                step(phc, General{}, zb + decltype(phc)::value, AnySB{});
            });
    };
    if (zero_halo)
        sweep(std::integral_constant<bool, true>{});
    else
        sweep(std::integral_constant<bool, false>{});
}

// Workgroups are dealt to the XCDs round-robin in launch order and each XCD
// has its own L2.  Renumber so that every XCD takes one contiguous run of
// (diamond, x-chunk) tiles: the x chunks of a diamond, whose redundant halo
// columns overlap, and neighbouring diamonds, which share edge rows, then
// read those cells through the same L2.  (A bijection for any XCD count; the
// count only sets the locality.)
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t launch_id, uint32_t n_tiles) {
    constexpr uint32_t NXCD = 8;
    const uint32_t per_xcd = n_tiles / NXCD, extra = n_tiles % NXCD;
    const uint32_t xcd = launch_id % NXCD, pos = launch_id / NXCD;
    return (xcd < extra ? xcd * (per_xcd + 1) : extra * (per_xcd + 1) + (xcd - extra) * per_xcd) + pos;
}

// Dependency-driven sweep (paper, Section "Runtime system": tiles are handed
// to thread groups as their dependencies are met, with no barrier between
// diamond rows).  One launch holds one workgroup per tile of every row, in
// row order; within a row the tiles are numbered as in the row launches
// (XCD-contiguous runs; each row's workgroups are padded to a multiple of
// the XCD count, so a workgroup lands on the same XCD as in a row launch).
// The hardware dispatches workgroups in launch order as compute units free
// up; a tile then waits until the tiles of the previous row whose cells it
// reads, or whose reads its stores would overwrite, are done: the two
// diamonds of row r-1 over its rows and the x chunks within kx of its own.
// Every tile a tile waits for comes earlier in the launch, so it has been
// dispatched and waits only on tiles earlier still: the earliest unfinished
// tile always runs, and the waits end.  They are bounded all the same: a
// wait gives up after spin_limit polls (at once once another one has),
// records the failure in *error for the host and lets the tile run, so
// every workgroup exits.
struct SweepSched {
    uint32_t* done;        // completion marks: row r's tile u at [(r % 4) * tpr + u]
    uint32_t* error;       // set nonzero when a wait gave up
    uint32_t base;         // mark of a finished row-r tile: base + r + 1 (monotone across runs)
    uint32_t spin_limit;   // polls before a wait gives up
    int32_t n_chunks, tpr, kx, H;
    int32_t nd[2];         // diamonds per row, by row parity
    int32_t nb[2];         // workgroups per row (tiles padded to a multiple of 8), by row parity
    int32_t clip_lo, clip_hi;   // rows outside [clip_lo, clip_hi) run the clipped-slot body
};

template <typename Real>
struct MwdSweepArgs {
    MwdArgs<Real> rows[2];   // the arguments of the even and of the odd rows (t_c aside)
    SweepSched s;
};

template <class S, typename Real, int DW, int VX, int WX, int NF, int NSC, int SY = 0>
__global__ void __launch_bounds__(64 * (DW / 2) * WX)
mwd_sweep_kernel(MwdSweepArgs<Real> sa) {
    using KK = MwdKernel<S, Real, DW, VX, WX, NF>;
    __shared__ Real stage[KK::LDS_ROWS * KK::SROW];
    __shared__ uint32_t sync_flags[SY ? 32 : 1];
    const SweepSched& sc = sa.s;
    // row and workgroup within the row (rows alternate two sizes)
    const int bid = (int)blockIdx.x, two = sc.nb[0] + sc.nb[1];
    const int rem = bid % two;
    const int r = 2 * (bid / two) + (rem >= sc.nb[0] ? 1 : 0);
    const int local = rem >= sc.nb[0] ? rem - sc.nb[0] : rem;
    const int n_tiles = sc.nd[r & 1] * sc.n_chunks;
    if (local >= n_tiles) return;   // padding
    const int u = (int)xcd_contiguous((uint32_t)local, (uint32_t)n_tiles);
    const int chunk = u % sc.n_chunks, diamond = u / sc.n_chunks;
    if (threadIdx.x == 0 && r > 0) {
        // row r-1's diamonds over this tile's rows: the row centres are
        // offset by half a diamond, up for odd rows, down for even ones
        const int m_lo = (r & 1) ? diamond : diamond - 1;
        const int nd_prev = sc.nd[(r - 1) & 1];
        const uint32_t want = sc.base + (uint32_t)r;   // mark of a finished row-(r-1) tile
        const uint32_t* row_done = sc.done + ((r - 1) % 4) * sc.tpr;
        uint32_t spins = 0;
        for (int m = m_lo; m <= m_lo + 1; ++m) {
            if (m < 0 || m >= nd_prev) continue;
            for (int c = chunk - sc.kx; c <= chunk + sc.kx; ++c) {
                if (c < 0 || c >= sc.n_chunks) continue;
                const uint32_t* f = row_done + m * sc.n_chunks + c;
                // relaxed device-scope polls read the mark from memory (not a
                // stale L2 copy) without invalidating the caches each time
                while ((int32_t)(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - want) < 0) {
                    if (spins++ >= sc.spin_limit ||
                        __hip_atomic_load(sc.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        __hip_atomic_store(sc.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
        }
        // one acquire for all the marks read
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // Thread 0's acquire invalidated the CU's and the XCD's caches,
    // which all waves of the workgroup read through: after the barrier every
    // wave sees what the tiles waited for wrote.  (One invalidation per tile:
    // an acquire in every wave would also drop the cached data of the other
    // tiles running on the XCD, a dozen times per tile.)
    __syncthreads();
    // (the arguments stay in the kernel's argument segment, where the
    // compiler reloads them instead of holding them in registers)
    const MwdArgs<Real>& a = sa.rows[r & 1];
    const int64_t t_c = (int64_t)r * sc.H;
    if constexpr (NSC > 0) {
        if (r < sc.clip_lo || r >= sc.clip_hi)
            mwd_tile<S, Real, DW, VX, WX, NSC, NF, SY>(a, t_c, chunk, diamond, stage, sync_flags);
        else
            mwd_tile<S, Real, DW, VX, WX, 0, NF, SY>(a, t_c, chunk, diamond, stage, sync_flags);
    } else {
        mwd_tile<S, Real, DW, VX, WX, 0, NF, SY>(a, t_c, chunk, diamond, stage, sync_flags);
    }
    // The barrier waits until every wave's stores have reached the XCD's L2;
    // thread 0's releasing store then writes the L2 back to memory before
    // the mark, so the tile's results are visible device-wide once it is
    // marked done.
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(sc.done + (r % 4) * sc.tpr + u, sc.base + (uint32_t)r + 1u, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// One diamond row: one workgroup per (diamond, x-chunk) tile.
template <class S, typename Real, int DW, int VX, int WX, int NSV, int NF, int SY = 0>
__global__ void __launch_bounds__(64 * (DW / 2) * WX)
mwd_row_kernel(MwdArgs<Real> a) {
    using KK = MwdKernel<S, Real, DW, VX, WX, NF>;
    __shared__ Real stage[KK::LDS_ROWS * KK::SROW];
    __shared__ uint32_t sync_flags[SY ? 32 : 1];
    const uint32_t tile = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    mwd_tile<S, Real, DW, VX, WX, NSV, NF, SY>(a, a.t_c, (int)(tile % gridDim.x), (int)(tile / gridDim.x), stage,
                                               sync_flags);
}

}  // namespace girih
