/*
 * Reference sweep for the paper's stencils — TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle: a plain, slow, obviously correct CPU implementation
 * of what the blocked GPU sweep must reproduce.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * source with the GPU library.
 *
 * What it computes (paper, Section "Background / Cache blocking", and the
 * captions of Listings 1-4): the naive schedule.  For t = 0..T-1, every
 * interior point (k,j,i) of U is set from V by the stencil formula, then the
 * two arrays swap roles.  Halo cells (width h) are fixed Dirichlet values and
 * are never written.  After T steps the result is the interior of buffer T%2.
 *
 * Evaluation order: C's left-to-right parse of each listing, round-to-nearest
 * IEEE arithmetic, no contraction into fused multiply-add (build with
 * -ffp-contract=off).  Per stencil:
 *   7c  (Listing 1): ((c0*V + c1*(V[i+1]+V[i-1])) + c1*(V[j+1]+V[j-1]))
 *                     + c1*(V[k+1]+V[k-1])
 *   7v  (Listing 2): C0*V + C1*V[i+1] + C2*V[i-1] + C3*V[j+1] + C4*V[j-1]
 *                     + C5*V[k+1] + C6*V[k-1], accumulated left to right
 *   25c (Listing 3, bracketed term only, i.e. the first-order-in-time Jacobi
 *        form): c0*V + c1*S1 + c2*S2 + c3*S3 + c4*S4, left to right, with
 *        S_r = V[i+r]+V[i-r]+V[j+r]+V[j-r]+V[k+r]+V[k-r], left to right
 *   25v (Listing 4): C00*V + C01*(V[i+1]+V[i-1]) + C02*(V[j+1]+V[j-1])
 *                     + C03*(V[k+1]+V[k-1]) + C04*(x, r=2) + ... + C12*(z, r=4),
 *        accumulated left to right
 *   25l (Listing 3 as printed, second order in time):
 *        (2*V - U) + C*(c0*V + c1*S1 + c2*S2 + c3*S3 + c4*S4), where U is the
 *        value the point holds in the array being overwritten, i.e. time
 *        level t-1; buf1 therefore holds u^{-1} on entry, not a copy of the
 *        halo only.  One coefficient array C and five constants.
 *   27b (the 27-point box stencil of Section "Handling other stencil types",
 *        constant coefficients by distance class; the paper prints no
 *        listing for it, so the order is this file's):
 *        ((c0*V + c1*F) + c2*E) + c3*K, where F, E and K sum the 6 face, 12
 *        edge and 8 corner neighbours, each in lexicographic order of the
 *        offset (dk, dj, di), components -1 < 0 < +1, dk slowest.
 *
 * Array layout (Listings 1-4 index U[k][j][i], i fastest): element (k,j,i),
 * with k in [-h, nz+h), j in [-h, ny+h), i in [-h, nx+h), lives at
 * ((k+h)*pitch_y + (j+h))*pitch_x + (i+h).  Coefficient arrays use the same
 * layout; their halo is never read.
 */
#include <stddef.h>
#include <stdint.h>

#define ST_7C 0
#define ST_7V 1
#define ST_25C 2
#define ST_25V 3
#define ST_25L 4
#define ST_27B 5

#define IDX(k, j, i) ((((int64_t)(k) + h) * pitch_y + ((int64_t)(j) + h)) * pitch_x + ((int64_t)(i) + h))

/* One Jacobi step of each stencil: U <- F(V).  Written once per precision
 * through a macro so that float and double follow the same text. */
#define DEFINE_STEP(REAL, SUFFIX)                                                        \
static void step_##SUFFIX(int stencil, int64_t nx, int64_t ny, int64_t nz, int64_t h,    \
                          int64_t pitch_x, int64_t pitch_y, REAL *U, const REAL *V,      \
                          const REAL *c, const REAL *const *C)                           \
{                                                                                        \
    int64_t k;                                                                           \
    _Pragma("omp parallel for schedule(static)")                                         \
    for (k = 0; k < nz; k++) {                                                           \
        for (int64_t j = 0; j < ny; j++) {                                               \
            for (int64_t i = 0; i < nx; i++) {                                           \
                const int64_t p = IDX(k, j, i);                                          \
                REAL u;                                                                  \
                if (stencil == ST_7C) {                                                  \
                    u = c[0] * V[p]                                                      \
                      + c[1] * (V[IDX(k, j, i + 1)] + V[IDX(k, j, i - 1)])               \
                      + c[1] * (V[IDX(k, j + 1, i)] + V[IDX(k, j - 1, i)])               \
                      + c[1] * (V[IDX(k + 1, j, i)] + V[IDX(k - 1, j, i)]);              \
                } else if (stencil == ST_7V) {                                           \
                    u = C[0][p] * V[p]                                                   \
                      + C[1][p] * V[IDX(k, j, i + 1)]                                    \
                      + C[2][p] * V[IDX(k, j, i - 1)]                                    \
                      + C[3][p] * V[IDX(k, j + 1, i)]                                    \
                      + C[4][p] * V[IDX(k, j - 1, i)]                                    \
                      + C[5][p] * V[IDX(k + 1, j, i)]                                    \
                      + C[6][p] * V[IDX(k - 1, j, i)];                                   \
                } else if (stencil == ST_25C) {                                          \
                    u = c[0] * V[p];                                                     \
                    for (int r = 1; r <= 4; r++) {                                       \
                        REAL s = V[IDX(k, j, i + r)] + V[IDX(k, j, i - r)]               \
                               + V[IDX(k, j + r, i)] + V[IDX(k, j - r, i)]               \
                               + V[IDX(k + r, j, i)] + V[IDX(k - r, j, i)];              \
                        u = u + c[r] * s;                                                \
                    }                                                                    \
                } else if (stencil == ST_27B) {                                          \
                    REAL f = 0, e = 0, q = 0;                                            \
                    int nf = 0, ne = 0, nq = 0;                                          \
                    for (int dk = -1; dk <= 1; dk++)                                     \
                        for (int dj = -1; dj <= 1; dj++)                                 \
                            for (int di = -1; di <= 1; di++) {                           \
                                const int m = (dk != 0) + (dj != 0) + (di != 0);         \
                                const REAL v = V[IDX(k + dk, j + dj, i + di)];           \
                                if (m == 1) { f = nf++ ? f + v : v; }                    \
                                else if (m == 2) { e = ne++ ? e + v : v; }               \
                                else if (m == 3) { q = nq++ ? q + v : v; }               \
                            }                                                            \
                    u = c[0] * V[p] + c[1] * f + c[2] * e + c[3] * q;                    \
                } else if (stencil == ST_25L) {                                          \
                    REAL b = c[0] * V[p];                                                \
                    for (int r = 1; r <= 4; r++) {                                       \
                        REAL s = V[IDX(k, j, i + r)] + V[IDX(k, j, i - r)]               \
                               + V[IDX(k, j + r, i)] + V[IDX(k, j - r, i)]               \
                               + V[IDX(k + r, j, i)] + V[IDX(k - r, j, i)];              \
                        b = b + c[r] * s;                                                \
                    }                                                                    \
                    u = 2 * V[p] - U[p] + C[0][p] * b;                                   \
                } else {                                                                 \
                    u = C[0][p] * V[p];                                                  \
                    for (int r = 1; r <= 4; r++) {                                       \
                        u = u + C[3 * r - 2][p] * (V[IDX(k, j, i + r)] + V[IDX(k, j, i - r)]); \
                        u = u + C[3 * r - 1][p] * (V[IDX(k, j + r, i)] + V[IDX(k, j - r, i)]); \
                        u = u + C[3 * r][p] * (V[IDX(k + r, j, i)] + V[IDX(k - r, j, i)]);     \
                    }                                                                    \
                }                                                                        \
                U[p] = u;                                                                \
            }                                                                            \
        }                                                                                \
    }                                                                                    \
}                                                                                        \
                                                                                         \
int oracle_sweep_##SUFFIX(int stencil, int64_t nx, int64_t ny, int64_t nz, int64_t h,    \
                          int64_t pitch_x, int64_t pitch_y, REAL *buf0, REAL *buf1,      \
                          const REAL *const_coefs, const REAL *const *coef_arrays,       \
                          int64_t T)                                                     \
{                                                                                        \
    const int64_t R = (stencil == ST_7C || stencil == ST_7V || stencil == ST_27B) ? 1 : 4; \
    if (stencil < 0 || stencil > 5) return -1;                                           \
    if (nx < 0 || ny < 0 || nz < 0 || T < 0 || h != R) return -1;                        \
    if (pitch_x < nx + 2 * h || pitch_y < ny + 2 * h) return -1;                         \
    REAL *V = buf0, *U = buf1;                                                           \
    for (int64_t t = 0; t < T; t++) {                                                    \
        step_##SUFFIX(stencil, nx, ny, nz, h, pitch_x, pitch_y, U, V,                    \
                      const_coefs, coef_arrays);                                         \
        REAL *tmp = U; U = V; V = tmp;                                                   \
    }                                                                                    \
    return 0;                                                                            \
}

DEFINE_STEP(double, f64)
DEFINE_STEP(float, f32)

/* Number of OpenMP threads the sweep will use (1 when built without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_num_threads(int n) { (void)n; }
#endif
