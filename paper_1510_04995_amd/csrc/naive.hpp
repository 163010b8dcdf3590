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
#include <type_traits>

#include "lanes.hpp"
#include "stencils.hpp"

namespace girih {

// Compile-time loop: f(std::integral_constant<int, I>) for I = B..E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for_n(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for_n<B + 1, E>(f);
    }
}

template <typename Real>
struct NaiveArgs {
    GridDesc g;
    const Real* V;    // time level t
    Real* U;          // time level t+1
    CoefArgs<Real> coef;
    int32_t z_chunk;
    int32_t xcd_runs;   // variant 1: 1 = renumber blocks into XCD-contiguous runs
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
        if constexpr (S::LEAPFROG) n.uo = U[p];   // time level t-1, about to be overwritten
        U[p] = S::apply(n, a.coef.k, cf);
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) w[m] = w[m + 1];
    }
}

// The 27-point box stencil: the same march along z, each lane keeping the
// 3x3 columns around its own for the planes z-1, z, z+1 in registers (nine
// loads per plane, the eight beside its own column shared with neighbouring
// lanes and rows through the caches).
template <typename Real>
__global__ void __launch_bounds__(256)
naive_box_kernel(NaiveArgs<Real> a) {
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
    // w[d][c]: plane z-1+d, column c = (dy+1)*3 + (dx+1)
    Real w[3][9];
    int64_t p = g.idx(z0, y, x);
    auto load_plane = [&](Real (&dst)[9], int64_t q) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) dst[(dy + 1) * 3 + dx + 1] = V[q + dy * px + dx];
    };
    load_plane(w[0], p - plane);
    load_plane(w[1], p);
    for (int64_t z = z0; z < z1; ++z, p += plane) {
        load_plane(w[2], p + plane);
        Box27<Real> b;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 9; ++c) b.v[d * 9 + c] = w[d][c];
        U[p] = Stencil27B::apply_box(b, a.coef.k);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            w[0][c] = w[1][c];
            w[1][c] = w[2][c];
        }
    }
}

// Box stencil, variant 1: register columns, no LDS and no barriers.  A wave
// holds 64 consecutive x cells (x0 - 1 .. x0 + 62) of KY + 2 rows along y
// (y0 - 1 .. y0 + KY) for the planes z - 1, z, z + 1, and marches z over its
// chunk reading one new plane (KY + 2 coalesced rows) per step, one step
// ahead.  The x - 1 and x + 1 values of a new plane come from the
// neighbouring lanes (two DPP moves per row) and are kept with it, so an
// update reads all 27 operands from registers.  Lanes 0 and 63 only load
// (their outer neighbour is in no register): each wave stores 62 x cells of
// KY rows.  Blocks are 64 x W threads; the grid is ceil(nx / 62) x
// ceil(ny / (W KY)) x z chunks, renumbered into XCD-contiguous runs as in the
// plane-tile kernel (the y halo rows of a block are its neighbours' rows).
template <typename Real, int KY>
__global__ void __launch_bounds__(256)
naive_box_cols_kernel(NaiveArgs<Real> a) {
    constexpr int NR = KY + 2;   // rows a lane holds per plane
    const GridDesc& g = a.g;
    const int lane = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const uint32_t NXCD = a.xcd_runs ? 8u : 1u;
    const uint32_t gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
    const uint32_t lid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t per_xcd = nb / NXCD, extra = nb % NXCD, xcd = lid % NXCD, pos = lid / NXCD;
    const uint32_t tid_run = (xcd < extra ? xcd * (per_xcd + 1) : extra * (per_xcd + 1) + (xcd - extra) * per_xcd) + pos;
    const uint32_t bx = tid_run % gx, by = (tid_run / gx) % gy, bz = tid_run / (gx * gy);
    const int64_t y0 = ((int64_t)by * blockDim.y + wave) * KY;
    const int64_t z0 = (int64_t)bz * a.z_chunk;
    int64_t z1 = z0 + a.z_chunk;
    if (z1 > g.nz) z1 = g.nz;
    // both conditions are uniform across the wave, and nothing below waits
    // on other waves
    if (y0 >= g.ny || z0 >= z1) return;
    const int64_t x = (int64_t)bx * 62 + lane - 1;
    // rows and columns clamped into the haloed box (cells past it belong to
    // no stored neighbourhood)
    const int64_t xc = x < -1 ? -1 : (x > g.nx ? g.nx : x);
    const bool st_x = lane >= 1 && lane <= 62 && x < g.nx;
    const int64_t plane = g.plane();
    // per-lane element offsets of the rows (row y0 - 1 + r clamped to the
    // halo row ny) in plane -h: kept in registers across the sweep, which
    // measured faster here than a wave-uniform row offset plus a lane offset
    // recomputed at every access (278 against 242 GLUP/s in FP64)
    int64_t ro[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int64_t yr = y0 - 1 + r > g.ny ? g.ny : y0 - 1 + r;
        ro[r] = g.idx(-g.h, yr, xc);
    }
    const Real* __restrict__ V = a.V;
    Real* __restrict__ U = a.U;
    // planes z - 1, z, z + 1 at ring slots (ph, ph + 1, ph + 2) mod 3: the
    // lane's own value (c) and those of x - 1 (l) and x + 1 (r)
    Real c[3][NR], l[3][NR], r[3][NR], nxt[NR];
    auto load = [&](Real (&d)[NR], int64_t q) __attribute__((always_inline)) {
        const int64_t off = (q + g.h) * plane;
#pragma unroll
        for (int k = 0; k < NR; ++k) d[k] = V[off + ro[k]];
    };
    auto insert = [&](int s, const Real (&v)[NR]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            c[s][k] = v[k];
            l[s][k] = lane_shift<0x138>(v[k]);
            r[s][k] = lane_shift<0x130>(v[k]);
        }
    };
    load(nxt, z0 - 1);
    insert(0, nxt);
    load(nxt, z0);
    insert(1, nxt);
    load(nxt, z0 + 1);
    auto step = [&](auto phc, int64_t z) __attribute__((always_inline)) {
        constexpr int ph = decltype(phc)::value;
        constexpr int s2 = (ph + 2) % 3;
        insert(s2, nxt);
        if (z + 1 < z1) load(nxt, z + 2);   // plane z + 2 <= nz: inside the haloed box
        const int64_t off = (z + g.h) * plane;
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            Box27<Real> b;
#pragma unroll
            for (int m = 0; m < 27; ++m) {
                const int dz = m / 9 - 1, dy = (m / 3) % 3 - 1, dx = m % 3 - 1;
                const int s = (ph + 1 + dz + 3) % 3, row = k + 1 + dy;
                b.v[m] = dx < 0 ? l[s][row] : (dx > 0 ? r[s][row] : c[s][row]);
            }
            const Real u = Stencil27B::apply_box(b, a.coef.k);
            if (st_x && y0 + k < g.ny) U[off + ro[k + 1]] = u;
        }
    };
    for (int64_t z = z0; z < z1; z += 3) {
        step(std::integral_constant<int, 0>{}, z);
        if (z + 1 < z1) step(std::integral_constant<int, 1>{}, z + 1);
        if (z + 2 < z1) step(std::integral_constant<int, 2>{}, z + 2);
    }
}

// Star stencils with constant coefficients, variant 2: register columns, no
// LDS and no barriers.  A wave holds 64 consecutive x cells (x0 - R ..
// x0 + 63 - R) of KY rows (y0 .. y0 + KY - 1) for the 2R + 1 planes of their
// z-window, and the 2R rows beside them (y0 - R .. y0 - 1, y0 + KY ..
// y0 + KY + R - 1) of the centre plane.  Per z step it loads one new plane of
// its rows and the side rows of the next centre plane, both one step ahead;
// the x neighbours are the neighbouring lanes' centre values (r chained DPP
// moves reach x + r), so lanes 0 .. R-1 and 64-R .. 63 only load and each
// wave stores 64 - 2R x cells of KY rows.  Blocks are 64 x W threads on a
// grid of ceil(nx / (64 - 2R)) x ceil(ny / (W KY)) x z chunks, numbered in
// XCD-contiguous runs.
template <class S, typename Real, int KY>
__global__ void __launch_bounds__(256)
naive_star_cols_kernel(NaiveArgs<Real> a) {
    constexpr int R = S::R, NZ = 2 * R + 1, OWN = 64 - 2 * R;
    static_assert(S::NCOEF == 0 && !S::LEAPFROG && !S::BOX, "constant-coefficient star stencils");
    const GridDesc& g = a.g;
    const int lane = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const uint32_t NXCD = a.xcd_runs ? 8u : 1u;
    const uint32_t gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
    const uint32_t lid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t per_xcd = nb / NXCD, extra = nb % NXCD, xcd = lid % NXCD, pos = lid / NXCD;
    const uint32_t tid_run = (xcd < extra ? xcd * (per_xcd + 1) : extra * (per_xcd + 1) + (xcd - extra) * per_xcd) + pos;
    const uint32_t bx = tid_run % gx, by = (tid_run / gx) % gy, bz = tid_run / (gx * gy);
    const int64_t y0 = ((int64_t)by * blockDim.y + wave) * KY;
    const int64_t z0 = (int64_t)bz * a.z_chunk;
    int64_t z1 = z0 + a.z_chunk;
    if (z1 > g.nz) z1 = g.nz;
    // uniform across the wave; nothing below waits on other waves
    if (y0 >= g.ny || z0 >= z1) return;
    const int64_t x = (int64_t)bx * OWN + lane - R;
    // rows and columns clamped into the haloed box (cells past it belong to
    // no stored neighbourhood)
    const int64_t xc = x >= g.nx + R ? g.nx + R - 1 : x;   // x >= -R always
    const bool st_x = lane >= R && lane < 64 - R && x < g.nx;
    auto clampy = [&](int64_t y) { return y < -R ? -R : (y > g.ny + R - 1 ? g.ny + R - 1 : y); };
    const int64_t plane = g.plane();
    // addresses: a row's element offset (uniform across the wave, so held in
    // scalar registers) plus the lane's byte offset within the row
    const uint32_t xb = (uint32_t)((xc + g.h) * (int64_t)sizeof(Real));
    auto row_off = [&](int64_t y) { return (clampy(y) + g.h) * g.pitch_x; };
    auto at = [&](const Real* base) -> const Real& {
        return *reinterpret_cast<const Real*>(reinterpret_cast<const char*>(base) + xb);
    };
    const Real* __restrict__ V = a.V;
    Real* __restrict__ U = a.U;
    // z-window of the own rows: plane z + d at slot (ph + R + d) mod NZ
    Real w[NZ][KY], nxt[KY], side[2 * R], snx[2 * R];
    auto load_rows = [&](Real (&d)[KY], int64_t q) __attribute__((always_inline)) {
        const Real* pb = V + (q + g.h) * plane;
#pragma unroll
        for (int k = 0; k < KY; ++k) d[k] = at(pb + row_off(y0 + k));
    };
    // side rows y0 - R .. y0 - 1 (index i < R) and y0 + KY .. y0 + KY + R - 1
    auto load_side = [&](Real (&d)[2 * R], int64_t q) __attribute__((always_inline)) {
        const Real* pb = V + (q + g.h) * plane;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            d[i] = at(pb + row_off(y0 - R + i));
            d[R + i] = at(pb + row_off(y0 + KY + i));
        }
    };
    // planes z0 - R .. z0 + R - 1 (inside the haloed box: z0 >= 0, z0 + R - 1 < nz + R)
    static_for_n<0, 2 * R>([&](auto dc) __attribute__((always_inline)) {
        constexpr int d = decltype(dc)::value;
        load_rows(w[d], z0 - R + d);
    });
    load_rows(nxt, z0 + R);
    load_side(snx, z0);
    auto step = [&](auto phc, int64_t z) __attribute__((always_inline)) {
        constexpr int ph = decltype(phc)::value;
        // plane z + R enters the window; the side rows of plane z become current
#pragma unroll
        for (int k = 0; k < KY; ++k) w[(ph + 2 * R) % NZ][k] = nxt[k];
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) side[i] = snx[i];
        if (z + 1 < z1) {
            load_rows(nxt, z + 1 + R);   // <= z1 - 1 + R < nz + R
            load_side(snx, z + 1);
        }
        Real* const ub = U + (z + g.h) * plane;
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            Nbhd<Real, R> n;
            n.c = w[(ph + R) % NZ][k];
            Real xp = n.c, xm = n.c;
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                xp = lane_shift<0x130>(xp);
                xm = lane_shift<0x138>(xm);
                n.xp[r - 1] = xp;
                n.xm[r - 1] = xm;
                n.zp[r - 1] = w[(ph + R + r) % NZ][k];
                n.zm[r - 1] = w[(ph + R - r) % NZ][k];
                n.yp[r - 1] = k + r < KY ? w[(ph + R) % NZ][k + r] : side[R + k + r - KY];
                n.ym[r - 1] = k - r >= 0 ? w[(ph + R) % NZ][k - r] : side[R + k - r];
            }
            const Real u = S::apply(n, a.coef.k, static_cast<const Real*>(nullptr));
            if (st_x && y0 + k < g.ny)
                *reinterpret_cast<Real*>(reinterpret_cast<char*>(ub + row_off(y0 + k)) + xb) = u;
        }
    };
    for (int64_t z = z0; z < z1; z += NZ) {
        static_for_n<0, NZ>([&](auto phc) __attribute__((always_inline)) {
            if (z + decltype(phc)::value < z1) step(phc, z + decltype(phc)::value);
        });
    }
}

// Variant 1: the same sweep with the x/y neighbours of each plane taken from
// an LDS tile.  A block of 64 x BY threads marches z as above; at every plane
// it stages the (BY + 2R) x (64 + 2R) tile of V around its columns: each
// thread writes its own centre value from its z-window, and the halo rows and
// columns come from memory once per block.  With BY rows per block the y
// halo is read 2R/BY times per update instead of 2R/4 times through the
// caches, which matters for R = 4.
template <class S, typename Real, int BY>
__global__ void __launch_bounds__(64 * BY)
naive_tile_kernel(NaiveArgs<Real> a) {
    constexpr int R = S::R, BX = 64, TX = BX + 2 * R, TY = BY + 2 * R;
    constexpr int NHALO = 2 * R * TX + 2 * R * BY;   // halo cells of the tile
    __shared__ Real tile[TY][TX];
    const GridDesc& g = a.g;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
    // Blocks are dealt to the XCDs round-robin in launch order and each XCD
    // has its own L2: with xcd_runs, renumber them so that every XCD sweeps
    // one contiguous run of tiles (x fastest, then y, then z chunks); a tile's
    // halo rows and columns, read from its neighbours' cells, then come
    // through the same L2.  (The host turns it off where many coefficient
    // streams make the launch-order interleaving the faster one.)
    const uint32_t NXCD = a.xcd_runs ? 8u : 1u;
    const uint32_t gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
    const uint32_t lid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t per_xcd = nb / NXCD, extra = nb % NXCD, xcd = lid % NXCD, pos = lid / NXCD;
    const uint32_t tid_run = (xcd < extra ? xcd * (per_xcd + 1) : extra * (per_xcd + 1) + (xcd - extra) * per_xcd) + pos;
    const uint32_t bx = tid_run % gx, by = (tid_run / gx) % gy, bz = tid_run / (gx * gy);
    const int64_t x0 = (int64_t)bx * BX, y0 = (int64_t)by * BY;
    const int64_t x = x0 + tx, y = y0 + ty;
    const bool mine = x < g.nx && y < g.ny;
    const int64_t z0 = (int64_t)bz * a.z_chunk;
    int64_t z1 = z0 + a.z_chunk;
    if (z1 > g.nz) z1 = g.nz;
    if (z0 >= z1) return;   // uniform across the block
    const int64_t plane = g.plane();
    const int64_t px = g.pitch_x;
    const Real* __restrict__ V = a.V;
    Real* __restrict__ U = a.U;
    // clamp into the haloed box: cells past it belong to no computed neighbourhood
    auto clampx = [&](int64_t v) { return v < -R ? -R : (v > g.nx + R - 1 ? g.nx + R - 1 : v); };
    auto clampy = [&](int64_t v) { return v < -R ? -R : (v > g.ny + R - 1 ? g.ny + R - 1 : v); };
    const int64_t xc = clampx(x), yc = clampy(y);
    Real w[2 * R + 1];
    int64_t p = g.idx(z0, yc, xc);
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) w[m] = V[p + (m - R) * plane];
    for (int64_t z = z0; z < z1; ++z, p += plane) {
        w[2 * R] = V[p + R * plane];
        tile[ty + R][tx + R] = w[R];
        for (int i = tid; i < NHALO; i += BX * BY) {
            int r, c;
            if (i < 2 * R * TX) {            // rows above and below the block
                const int k = i / TX;
                r = k < R ? k : BY + k;
                c = i % TX;
            } else {                          // columns left and right of it
                const int k = i - 2 * R * TX;
                r = R + k / (2 * R);
                const int cc = k % (2 * R);
                c = cc < R ? cc : BX + cc;
            }
            tile[r][c] = V[g.idx(z, clampy(y0 - R + r), clampx(x0 - R + c))];
        }
        __syncthreads();
        if (mine) {
            Nbhd<Real, R> n;
            n.c = w[R];
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                n.xp[r - 1] = tile[ty + R][tx + R + r];
                n.xm[r - 1] = tile[ty + R][tx + R - r];
                n.yp[r - 1] = tile[ty + R + r][tx + R];
                n.ym[r - 1] = tile[ty + R - r][tx + R];
                n.zp[r - 1] = w[R + r];
                n.zm[r - 1] = w[R - r];
            }
            Real cf[S::NCOEF > 0 ? S::NCOEF : 1];
#pragma unroll
            for (int m = 0; m < S::NCOEF; ++m) cf[m] = a.coef.arr[m][p];
            if constexpr (S::LEAPFROG) n.uo = U[p];   // time level t-1, about to be overwritten
        U[p] = S::apply(n, a.coef.k, cf);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) w[m] = w[m + 1];
    }
}

}  // namespace girih
