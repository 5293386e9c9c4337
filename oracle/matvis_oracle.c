/*
 * matvis_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the visibility-simulator hot path of
 * the matrix-based RIME paper (arXiv:2312.09763).  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it.  It shares no code, header or table with the
 * HIP library.
 *
 * Everything is double precision, written for readability rather than
 * speed: no blocking, no fusion, no reordering beyond what each definition
 * states.  OpenMP parallelises only independent outer loops.
 *
 * What is computed, and where the paper defines it:
 *   - unit vectors X_eq from (RA, Dec)                 Sec. 3.3, Eq. (xeq)
 *   - the rotation matrix R(t), with H = -LST           Sec. 3.3, Eq. (rotation)
 *   - X_hrz = R X_eq and the horizon cut U > 0          Sec. 3.3; Alg. 2 step (i)
 *   - beam values at the sources' (za, az)              Sec. 3.4; Alg. 2 step (ii)
 *   - the per-antenna matrix Z = sqrt(I) A F            Eq. (littlez); Alg. 2 (iii)-(iv)
 *   - the Gram matrix Z Z^H                              Eq. (zz); Alg. 2 step (v)
 *   - the end-to-end visibilities as a direct sum over
 *     sources for every antenna pair (not via Z)         Eq. (matvisrime), (matvisdelay)
 *   - the same direct sum for a polarised sky, with the
 *     brightness matrix built from I, Q, U, V            Sec. 2.1; Eq. (matvisrime)
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - the hour angle in Eq. (rotation) is H = -LST; with it R X_eq equals the
 *     textbook hour-angle (E, N, U) vector;
 *   - b_ij = x_i - x_j, as the fringe factorisation F_in F*_jn of Sec. 3.2 implies;
 *   - the horizon cut is strict (U > 0);
 *   - za = atan2(hypot(E, N), U), az = atan2(E, N) in [0, 2 pi), from North
 *     through East;
 *   - unpolarised sky: Z = sqrt(I) A F exactly as in Eq. (littlez), so a
 *     zenith source seen by a unit beam gives V = I;
 *   - grids: za_j = j dza (j < n_za, last row on the horizon), az_k = k daz,
 *     periodic in az.  Bilinear: za cell clamped to [0, n_za - 2].  Bicubic:
 *     Keys (1981) cubic convolution with a = -1/2 in index space, periodic in
 *     az, with Keys' ghost rows g[-1] = 3 g[0] - 3 g[1] + g[2] and
 *     g[n] = 3 g[n-1] - 3 g[n-2] + g[n-3] at the two za ends.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The arithmetic type.  The reference is built in double precision; a second
 * build with -DORC_REAL="long double" (x86 80-bit extended) runs the same
 * source in wider arithmetic, only to bound the double build's own rounding
 * on small cases.  Every array argument then has that type too. */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;
typedef ORC_REAL _Complex cplx;

#define SPEED_OF_LIGHT 299792458.0
/* pi to beyond long-double precision; in the double build this rounds to M_PI */
#define PI ((real)3.14159265358979323846264338327950288L)

int orc_version(void) { return 1; }

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. (xeq): X_eq = (cos a cos d, sin a cos d, sin d).  out is [n][3]. */
void orc_xeq(int64_t n, const real *ra, const real *dec, real *out) {
    for (int64_t i = 0; i < n; i++) {
        out[3 * i + 0] = cos(ra[i]) * cos(dec[i]);
        out[3 * i + 1] = sin(ra[i]) * cos(dec[i]);
        out[3 * i + 2] = sin(dec[i]);
    }
}

/* Eq. (rotation) with H = -lst and l = latitude; R is row-major [3][3]. */
void orc_rotation(real lst, real latitude, real *R) {
    real H = -lst;
    real l = latitude;
    R[0] = sin(H);
    R[1] = cos(H);
    R[2] = 0.0;
    R[3] = -sin(l) * cos(H);
    R[4] = sin(l) * sin(H);
    R[5] = cos(l);
    R[6] = cos(l) * cos(H);
    R[7] = -cos(l) * sin(H);
    R[8] = sin(l);
}

/* X_hrz = R X_eq for every source (Sec. 3.3).  xeq, xhrz are [n][3]. */
void orc_topocentric(const real *R, int64_t n, const real *xeq, real *xhrz) {
    for (int64_t i = 0; i < n; i++) {
        for (int r = 0; r < 3; r++) {
            real s = 0.0;
            for (int c = 0; c < 3; c++) s += R[3 * r + c] * xeq[3 * i + c];
            xhrz[3 * i + r] = s;
        }
    }
}

/* Horizon cut of Alg. 2 step (i): ascending indices of sources with U > 0. */
int64_t orc_visible(int64_t n, const real *xhrz, int32_t *idx) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (xhrz[3 * i + 2] > 0.0) idx[m++] = (int32_t)i;
    return m;
}

/* Zenith angle and azimuth (North through East) of topocentric unit vectors. */
void orc_azza(int64_t n, const real *xhrz, real *az, real *za) {
    for (int64_t i = 0; i < n; i++) {
        real e = xhrz[3 * i + 0], nn = xhrz[3 * i + 1], u = xhrz[3 * i + 2];
        za[i] = atan2(hypot(e, nn), u);
        real a = atan2(e, nn);
        if (a < 0.0) a += 2.0 * PI;
        if (a >= 2.0 * PI) a -= 2.0 * PI;
        az[i] = a;
    }
}

/* ---------------------------------------------------------------------- */
/* Beam interpolation on the az/za grid with the zenith as pole (Sec. 3.4) */
/* ---------------------------------------------------------------------- */

static int wrap(int k, int n) {
    int r = k % n;
    return r < 0 ? r + n : r;
}

/* Grid value with az wrapped periodically; za row must be in range. */
static cplx node(const cplx *g, int n_az, int j, int k) { return g[(int64_t)j * n_az + wrap(k, n_az)]; }

/* Bilinear interpolation of one complex grid plane g[n_za][n_az]. */
cplx orc_bilinear_one(const cplx *g, int n_za, int n_az, real dza, real daz, real za, real az) {
    real u = za / dza;
    real v = az / daz;
    int j0 = (int)floor(u);
    if (j0 < 0) j0 = 0;
    if (j0 > n_za - 2) j0 = n_za - 2;
    real t = u - j0;
    real kf = floor(v);
    real s = v - kf;
    int k0 = (int)kf;
    cplx a00 = node(g, n_az, j0, k0), a01 = node(g, n_az, j0, k0 + 1);
    cplx a10 = node(g, n_az, j0 + 1, k0), a11 = node(g, n_az, j0 + 1, k0 + 1);
    return (1.0 - t) * (1.0 - s) * a00 + (1.0 - t) * s * a01 + t * (1.0 - s) * a10 + t * s * a11;
}

/* Keys (1981) cubic-convolution kernel with a = -1/2. */
static real keys_w(real x) {
    const real a = -0.5;
    x = fabs(x);
    if (x <= 1.0) return (a + 2.0) * x * x * x - (a + 3.0) * x * x + 1.0;
    if (x < 2.0) return a * x * x * x - 5.0 * a * x * x + 8.0 * a * x - 4.0 * a;
    return 0.0;
}

/* Grid row j (possibly one of the two ghost rows) at column k. */
static cplx row_value(const cplx *g, int n_za, int n_az, int j, int k) {
    if (j == -1) return 3.0 * node(g, n_az, 0, k) - 3.0 * node(g, n_az, 1, k) + node(g, n_az, 2, k);
    if (j == n_za)
        return 3.0 * node(g, n_az, n_za - 1, k) - 3.0 * node(g, n_az, n_za - 2, k) + node(g, n_az, n_za - 3, k);
    return node(g, n_az, j, k);
}

/* Bicubic (Keys) interpolation of one complex grid plane g[n_za][n_az]. */
cplx orc_bicubic_one(const cplx *g, int n_za, int n_az, real dza, real daz, real za, real az) {
    real u = za / dza;
    real v = az / daz;
    int j0 = (int)floor(u);
    if (j0 < 0) j0 = 0;
    if (j0 > n_za - 2) j0 = n_za - 2;
    real t = u - j0;
    real kf = floor(v);
    real s = v - kf;
    int k0 = (int)kf;
    cplx acc = 0.0;
    for (int dj = -1; dj <= 2; dj++) {
        real wj = keys_w(t - dj);
        for (int dk = -1; dk <= 2; dk++) {
            real wk = keys_w(s - dk);
            acc += wj * wk * row_value(g, n_za, n_az, j0 + dj, k0 + dk);
        }
    }
    return acc;
}

/* Interpolate many points (Python-facing helper): mode 0 bilinear, 1 bicubic. */
void orc_interp(int mode, const cplx *g, int n_za, int n_az, real dza, real daz, int64_t n,
                const real *za, const real *az, cplx *out) {
    for (int64_t i = 0; i < n; i++)
        out[i] = mode == 0 ? orc_bilinear_one(g, n_za, n_az, dza, daz, za[i], az[i])
                           : orc_bicubic_one(g, n_za, n_az, dza, daz, za[i], az[i]);
}

/* ---------------------------------------------------------------------- */
/* Per-instance pieces                                                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t n_ant, n_feed, n_ax, n_beam;
    int32_t n_za, n_az;
    real dza, daz;
    real latitude;
    int32_t interp; /* 0 bilinear, 1 bicubic */
} orc_geom;

/* Visible set and beam values for one (t, nu).
 * beam_f: grid slice of channel f: [n_beam][n_feed][n_ax][n_za][n_az].
 * Outputs: idx[m], xhrz_vis[m][3], A[n_beam][n_feed][n_ax][m] (row stride n_src). */
static int64_t instance_sky(const orc_geom *G, real lst, int64_t n_src, const real *xeq, const cplx *beam_f,
                            int32_t *idx, real *xhrz_all, real *xhrz_vis, cplx *A) {
    real R[9];
    orc_rotation(lst, G->latitude, R);
    orc_topocentric(R, n_src, xeq, xhrz_all);
    int64_t m = orc_visible(n_src, xhrz_all, idx);
    int64_t plane = (int64_t)G->n_za * G->n_az;
    for (int64_t i = 0; i < m; i++) {
        const real *s = xhrz_all + 3 * (int64_t)idx[i];
        xhrz_vis[3 * i + 0] = s[0];
        xhrz_vis[3 * i + 1] = s[1];
        xhrz_vis[3 * i + 2] = s[2];
    }
    if (A) {
        for (int64_t i = 0; i < m; i++) {
            real az, za;
            orc_azza(1, xhrz_vis + 3 * i, &az, &za);
            for (int b = 0; b < G->n_beam; b++)
                for (int p = 0; p < G->n_feed; p++)
                    for (int k = 0; k < G->n_ax; k++) {
                        const cplx *g = beam_f + (((int64_t)b * G->n_feed + p) * G->n_ax + k) * plane;
                        cplx val = G->interp == 0 ? orc_bilinear_one(g, G->n_za, G->n_az, G->dza, G->daz, za, az)
                                                  : orc_bicubic_one(g, G->n_za, G->n_az, G->dza, G->daz, za, az);
                        A[(((int64_t)b * G->n_feed + p) * G->n_ax + k) * n_src + i] = val;
                    }
        }
    }
    return m;
}

/* Eq. (matvisrime) with C = diag(I, I) and the delay of Eq. (matvisdelay):
 *   V[a][b][p][q] = sum_{n visible} I_n sum_k A_{beam(a),p,k}(n) conj(A_{beam(b),q,k}(n))
 *                    * exp(-2 pi i nu (x_a - x_b) . s_n / c)
 * summed in ascending n, every (a, b) evaluated independently.
 * A is [n_beam][n_feed][n_ax][lda] over the m visible sources; flux_vis[m]. */
static void direct_sum(const orc_geom *G, const real *antpos, const int32_t *beam_idx, real freq, int64_t m,
                       const real *xhrz_vis, const real *flux_vis, const cplx *A, int64_t lda, cplx *V) {
    const int na = G->n_ant, nf = G->n_feed, nx = G->n_ax;
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < na; a++) {
        for (int b = 0; b < na; b++) {
            real bx = antpos[3 * a + 0] - antpos[3 * b + 0];
            real by = antpos[3 * a + 1] - antpos[3 * b + 1];
            real bz = antpos[3 * a + 2] - antpos[3 * b + 2];
            int ia = beam_idx ? beam_idx[a] : 0;
            int ib = beam_idx ? beam_idx[b] : 0;
            for (int p = 0; p < nf; p++)
                for (int q = 0; q < nf; q++) {
                    cplx acc = 0.0;
                    for (int64_t n = 0; n < m; n++) {
                        const real *s = xhrz_vis + 3 * n;
                        real tau = (bx * s[0] + by * s[1] + bz * s[2]) / SPEED_OF_LIGHT;
                        real ph = -2.0 * PI * freq * tau;
                        cplx fringe = cos(ph) + I * sin(ph);
                        cplx beams = 0.0;
                        for (int k = 0; k < nx; k++) {
                            cplx aa = A[(((int64_t)ia * nf + p) * nx + k) * lda + n];
                            cplx bb = A[(((int64_t)ib * nf + q) * nx + k) * lda + n];
                            beams += aa * conj(bb);
                        }
                        acc += flux_vis[n] * beams * fringe;
                    }
                    V[(((int64_t)a * na + b) * nf + p) * nf + q] = acc;
                }
        }
    }
}

/* End-to-end reference for a list of (t, f) instances.
 *   antpos [n_ant][3], beam_idx [n_ant] or NULL, freqs [n_freq], lsts [n_time],
 *   ra/dec [n_src], flux [n_freq][n_src],
 *   beam_grid [n_beam][n_freq][n_feed][n_ax][n_za][n_az] complex128,
 *   inst_t/inst_f [n_inst], V out [n_inst][n_ant][n_ant][n_feed][n_feed] complex128.
 * Returns 0, or -1 on allocation failure. */
int orc_simulate(const orc_geom *G, const real *antpos, const int32_t *beam_idx, const real *freqs,
                 int32_t n_freq, const real *lsts, int64_t n_src, const real *ra, const real *dec,
                 const real *flux, const cplx *beam_grid, int32_t n_inst, const int32_t *inst_t,
                 const int32_t *inst_f, cplx *V) {
    real *xeq = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xall = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xvis = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *fvis = malloc(sizeof(real) * (n_src ? n_src : 1));
    int32_t *idx = malloc(sizeof(int32_t) * (n_src ? n_src : 1));
    int64_t plane = (int64_t)G->n_za * G->n_az;
    int64_t per_freq = (int64_t)G->n_feed * G->n_ax * plane;
    cplx *A = malloc(sizeof(cplx) * (size_t)G->n_beam * G->n_feed * G->n_ax * (n_src ? n_src : 1));
    cplx *slice = malloc(sizeof(cplx) * (size_t)G->n_beam * per_freq);
    if (!xeq || !xall || !xvis || !fvis || !idx || !A || !slice) {
        free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A); free(slice);
        return -1;
    }
    orc_xeq(n_src, ra, dec, xeq);
    int64_t vsz = (int64_t)G->n_ant * G->n_ant * G->n_feed * G->n_feed;
    for (int32_t i = 0; i < n_inst; i++) {
        int t = inst_t[i], f = inst_f[i];
        for (int b = 0; b < G->n_beam; b++)
            memcpy(slice + b * per_freq, beam_grid + ((int64_t)b * n_freq + f) * per_freq, sizeof(cplx) * per_freq);
        int64_t m = instance_sky(G, lsts[t], n_src, xeq, slice, idx, xall, xvis, A);
        for (int64_t n = 0; n < m; n++) fvis[n] = flux[(int64_t)f * n_src + idx[n]];
        direct_sum(G, antpos, beam_idx, freqs[f], m, xvis, fvis, A, n_src, V + i * vsz);
    }
    free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A); free(slice);
    return 0;
}

/* The direct sum of Eq. (matvisrime) for a chosen list of antenna pairs only
 * (pair_a[j], pair_b[j]), j < n_pair: V[inst][j][p][q].  Same arithmetic as
 * orc_simulate, for checking single entries of large problems. */
int orc_simulate_pairs(const orc_geom *G, const real *antpos, const int32_t *beam_idx, const real *freqs,
                       int32_t n_freq, const real *lsts, int64_t n_src, const real *ra, const real *dec,
                       const real *flux, const cplx *beam_grid, int32_t n_inst, const int32_t *inst_t,
                       const int32_t *inst_f, int32_t n_pair, const int32_t *pair_a, const int32_t *pair_b,
                       cplx *V) {
    real *xeq = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xall = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xvis = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *fvis = malloc(sizeof(real) * (n_src ? n_src : 1));
    int32_t *idx = malloc(sizeof(int32_t) * (n_src ? n_src : 1));
    int64_t plane = (int64_t)G->n_za * G->n_az;
    int64_t per_freq = (int64_t)G->n_feed * G->n_ax * plane;
    cplx *A = malloc(sizeof(cplx) * (size_t)G->n_beam * G->n_feed * G->n_ax * (n_src ? n_src : 1));
    cplx *slice = malloc(sizeof(cplx) * (size_t)G->n_beam * per_freq);
    if (!xeq || !xall || !xvis || !fvis || !idx || !A || !slice) {
        free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A); free(slice);
        return -1;
    }
    orc_xeq(n_src, ra, dec, xeq);
    const int nf = G->n_feed, nx = G->n_ax;
    for (int32_t i = 0; i < n_inst; i++) {
        int t = inst_t[i], f = inst_f[i];
        for (int b = 0; b < G->n_beam; b++)
            memcpy(slice + b * per_freq, beam_grid + ((int64_t)b * n_freq + f) * per_freq, sizeof(cplx) * per_freq);
        int64_t m = instance_sky(G, lsts[t], n_src, xeq, slice, idx, xall, xvis, A);
        for (int64_t n = 0; n < m; n++) fvis[n] = flux[(int64_t)f * n_src + idx[n]];
        real freq = freqs[f];
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t j = 0; j < n_pair; j++) {
            int a = pair_a[j], b = pair_b[j];
            real bx = antpos[3 * a + 0] - antpos[3 * b + 0];
            real by = antpos[3 * a + 1] - antpos[3 * b + 1];
            real bz = antpos[3 * a + 2] - antpos[3 * b + 2];
            int ia = beam_idx ? beam_idx[a] : 0;
            int ib = beam_idx ? beam_idx[b] : 0;
            for (int p = 0; p < nf; p++)
                for (int q = 0; q < nf; q++) {
                    cplx acc = 0.0;
                    for (int64_t n = 0; n < m; n++) {
                        const real *s = xvis + 3 * n;
                        real tau = (bx * s[0] + by * s[1] + bz * s[2]) / SPEED_OF_LIGHT;
                        real ph = -2.0 * PI * freq * tau;
                        cplx fringe = cos(ph) + I * sin(ph);
                        cplx beams = 0.0;
                        for (int k = 0; k < nx; k++)
                            beams += A[(((int64_t)ia * nf + p) * nx + k) * n_src + n] *
                                     conj(A[(((int64_t)ib * nf + q) * nx + k) * n_src + n]);
                        acc += fvis[n] * beams * fringe;
                    }
                    V[(((int64_t)i * n_pair + j) * nf + p) * nf + q] = acc;
                }
        }
    }
    free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A); free(slice);
    return 0;
}

/* Same direct sum, with the beam supplied by the caller for every source
 * (A_all [n_beam][n_feed][n_ax][n_src] at this instance), e.g. an analytic
 * beam evaluated exactly.  One instance; returns the visible count. */
int64_t orc_simulate_given_beam(const orc_geom *G, const real *antpos, const int32_t *beam_idx, real freq,
                                real lst, int64_t n_src, const real *ra, const real *dec, const real *flux_f,
                                const cplx *A_all, cplx *V) {
    real *xeq = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xall = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xvis = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *fvis = malloc(sizeof(real) * (n_src ? n_src : 1));
    int32_t *idx = malloc(sizeof(int32_t) * (n_src ? n_src : 1));
    cplx *A = malloc(sizeof(cplx) * (size_t)G->n_beam * G->n_feed * G->n_ax * (n_src ? n_src : 1));
    if (!xeq || !xall || !xvis || !fvis || !idx || !A) {
        free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A);
        return -1;
    }
    orc_xeq(n_src, ra, dec, xeq);
    int64_t m = instance_sky(G, lst, n_src, xeq, NULL, idx, xall, xvis, NULL);
    int64_t comps = (int64_t)G->n_beam * G->n_feed * G->n_ax;
    for (int64_t c = 0; c < comps; c++)
        for (int64_t n = 0; n < m; n++) A[c * n_src + n] = A_all[c * n_src + idx[n]];
    for (int64_t n = 0; n < m; n++) fvis[n] = flux_f[idx[n]];
    direct_sum(G, antpos, beam_idx, freq, m, xvis, fvis, A, n_src, V);
    free(xeq); free(xall); free(xvis); free(fvis); free(idx); free(A);
    return m;
}

/* Polarised sky, Eq. (matvisrime) with the source brightness matrix of Sec. 2.1
 * written from the Stokes parameters,
 *   C = [[I + Q, U + iV], [U - iV, I - Q]]  (indices: the beam's E-field axes k, k'),
 *   V[a][b][p][q] = sum_{n visible} sum_{k,k'} A_{beam(a),p,k}(n) C_{kk'}(n) conj(A_{beam(b),q,k'}(n))
 *                    * exp(-2 pi i nu (x_a - x_b) . s_n / c),
 * summed in ascending n.  stokes is [4][n_freq][n_src] (I, Q, U, V per channel);
 * needs n_ax = 2.  n_pair < 0 evaluates every (a, b) into V[inst][a][b][p][q];
 * otherwise the listed pairs into V[inst][j][p][q].  Returns 0, -1 on
 * allocation failure, -2 when n_ax != 2. */
int orc_simulate_pol(const orc_geom *G, const real *antpos, const int32_t *beam_idx, const real *freqs,
                     int32_t n_freq, const real *lsts, int64_t n_src, const real *ra, const real *dec,
                     const real *stokes, const cplx *beam_grid, int32_t n_inst, const int32_t *inst_t,
                     const int32_t *inst_f, int32_t n_pair, const int32_t *pair_a, const int32_t *pair_b,
                     cplx *V) {
    if (G->n_ax != 2) return -2;
    const int64_t ns1 = n_src ? n_src : 1;
    real *xeq = malloc(sizeof(real) * 3 * ns1);
    real *xall = malloc(sizeof(real) * 3 * ns1);
    real *xvis = malloc(sizeof(real) * 3 * ns1);
    real *svis = malloc(sizeof(real) * 4 * ns1);
    int32_t *idx = malloc(sizeof(int32_t) * ns1);
    int64_t plane = (int64_t)G->n_za * G->n_az;
    int64_t per_freq = (int64_t)G->n_feed * G->n_ax * plane;
    cplx *A = malloc(sizeof(cplx) * (size_t)G->n_beam * G->n_feed * G->n_ax * ns1);
    cplx *slice = malloc(sizeof(cplx) * (size_t)G->n_beam * per_freq);
    if (!xeq || !xall || !xvis || !svis || !idx || !A || !slice) {
        free(xeq); free(xall); free(xvis); free(svis); free(idx); free(A); free(slice);
        return -1;
    }
    orc_xeq(n_src, ra, dec, xeq);
    const int na = G->n_ant, nf = G->n_feed, nx = G->n_ax;
    const int64_t npair = n_pair < 0 ? (int64_t)na * na : n_pair;
    for (int32_t i = 0; i < n_inst; i++) {
        int t = inst_t[i], f = inst_f[i];
        for (int b = 0; b < G->n_beam; b++)
            memcpy(slice + b * per_freq, beam_grid + ((int64_t)b * n_freq + f) * per_freq, sizeof(cplx) * per_freq);
        int64_t m = instance_sky(G, lsts[t], n_src, xeq, slice, idx, xall, xvis, A);
        for (int st = 0; st < 4; st++)
            for (int64_t n = 0; n < m; n++) svis[st * ns1 + n] = stokes[((int64_t)st * n_freq + f) * n_src + idx[n]];
        real freq = freqs[f];
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < npair; j++) {
            int a = n_pair < 0 ? (int)(j / na) : pair_a[j];
            int b = n_pair < 0 ? (int)(j % na) : pair_b[j];
            real bx = antpos[3 * a + 0] - antpos[3 * b + 0];
            real by = antpos[3 * a + 1] - antpos[3 * b + 1];
            real bz = antpos[3 * a + 2] - antpos[3 * b + 2];
            int ia = beam_idx ? beam_idx[a] : 0;
            int ib = beam_idx ? beam_idx[b] : 0;
            for (int p = 0; p < nf; p++)
                for (int q = 0; q < nf; q++) {
                    cplx acc = 0.0;
                    for (int64_t n = 0; n < m; n++) {
                        const real *s = xvis + 3 * n;
                        real tau = (bx * s[0] + by * s[1] + bz * s[2]) / SPEED_OF_LIGHT;
                        real ph = -2.0 * PI * freq * tau;
                        cplx fringe = cos(ph) + I * sin(ph);
                        real si = svis[n], sq = svis[ns1 + n], su = svis[2 * ns1 + n], sv = svis[3 * ns1 + n];
                        cplx C[2][2];
                        C[0][0] = si + sq;
                        C[0][1] = su + I * sv;
                        C[1][0] = su - I * sv;
                        C[1][1] = si - sq;
                        cplx beams = 0.0;
                        for (int k = 0; k < nx; k++)
                            for (int k2 = 0; k2 < nx; k2++)
                                beams += A[(((int64_t)ia * nf + p) * nx + k) * n_src + n] * C[k][k2] *
                                         conj(A[(((int64_t)ib * nf + q) * nx + k2) * n_src + n]);
                        acc += beams * fringe;
                    }
                    V[(((int64_t)i * npair + j) * nf + p) * nf + q] = acc;
                }
        }
    }
    free(xeq); free(xall); free(xvis); free(svis); free(idx); free(A); free(slice);
    return 0;
}

/* Step references used by per-kernel tests.
 *
 * orc_zmatrix: Eq. (littlez) / Alg. 2 steps (iii)-(iv) for one instance:
 *   Z[(a, p)][(n, k)] = sqrt(I_n) A_{beam(a), p, k}(n) exp(-2 pi i nu x_a . s_n / c)
 * over the m visible sources (given their X_hrz, flux and beam values A
 * [n_beam][n_feed][n_ax][lda]).  Z is [n_ant * n_feed][m * n_ax] row-major. */
void orc_zmatrix(const orc_geom *G, const real *antpos, const int32_t *beam_idx, real freq, int64_t m,
                 const real *xhrz_vis, const real *flux_vis, const cplx *A, int64_t lda, cplx *Z) {
    const int na = G->n_ant, nf = G->n_feed, nx = G->n_ax;
    int64_t ncol = m * nx;
    for (int a = 0; a < na; a++) {
        int ia = beam_idx ? beam_idx[a] : 0;
        for (int64_t n = 0; n < m; n++) {
            const real *s = xhrz_vis + 3 * n;
            real tau = (antpos[3 * a] * s[0] + antpos[3 * a + 1] * s[1] + antpos[3 * a + 2] * s[2]) / SPEED_OF_LIGHT;
            real ph = -2.0 * PI * freq * tau;
            cplx F = cos(ph) + I * sin(ph);
            for (int p = 0; p < nf; p++)
                for (int k = 0; k < nx; k++)
                    Z[((int64_t)a * nf + p) * ncol + n * nx + k] =
                        sqrt(flux_vis[n]) * A[(((int64_t)ia * nf + p) * nx + k) * lda + n] * F;
        }
    }
}

/* orc_gram: Eq. (zz), V = Z Z^H by its definition (every entry, both triangles).
 * Z is [nrow][ncol] complex128, V is [nrow][nrow]. */
void orc_gram(int64_t nrow, int64_t ncol, const cplx *Z, cplx *V) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrow; r++)
        for (int64_t c = 0; c < nrow; c++) {
            cplx acc = 0.0;
            for (int64_t k = 0; k < ncol; k++) acc += Z[r * ncol + k] * conj(Z[c * ncol + k]);
            V[r * nrow + c] = acc;
        }
}

/* Sky of one instance for step tests: visible indices, their X_hrz and the
 * beam at them.  Returns the visible count m. */
int64_t orc_instance_sky(const orc_geom *G, real lst, int64_t n_src, const real *ra, const real *dec,
                         const cplx *beam_f, int32_t *idx, real *xhrz_vis, cplx *A) {
    real *xeq = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    real *xall = malloc(sizeof(real) * 3 * (n_src ? n_src : 1));
    if (!xeq || !xall) {
        free(xeq); free(xall);
        return -1;
    }
    orc_xeq(n_src, ra, dec, xeq);
    int64_t m = instance_sky(G, lst, n_src, xeq, beam_f, idx, xall, xhrz_vis, A);
    free(xeq); free(xall);
    return m;
}
