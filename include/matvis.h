/*
 * matvis.h -- C ABI of the MI355X (gfx950) matrix-based visibility simulator.
 *
 * The library evaluates the point-source RIME of arXiv:2312.09763 the way its
 * Sec. 3.5 (Alg. 2) lays it out, for many (time, frequency) instances at once:
 *   (i)   rotate sources to topocentric ENU with R(t) of Eq. (rotation) and cut
 *         those at or below the horizon (U <= 0), order-preserving compaction;
 *   (ii)  interpolate the beam (Jones terms) at the visible sources' (za, az)
 *         on an az/za grid whose pole is the zenith (Sec. 3.4);
 *   (iii) antenna phase exp(-2 pi i nu x_a . s / c) (the fringe factorisation
 *         of Sec. 3.2), with FP64 range reduction of the argument;
 *   (iv)  Z[(a,p),(n,k)] = sqrt(I_n) A_{beam(a),p,k}(n) F_a(n)  (Eq. littlez);
 *   (v)   V = Z Z^H  (Eq. zz), lower-triangle tiles on MFMA, Hermitian fill.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (HIP global memory) unless the
 *     comment says host.  The caller owns every input and output buffer; the
 *     context owns all scratch.  No pointer is kept after a call returns
 *     except for the asynchronous use on `stream` (a hipStream_t passed as
 *     void*, NULL = the null stream) until the stream is synchronised.
 *   - Angles are radians, positions metres (ENU), frequencies Hz, fluxes Jy.
 *   - Complex numbers are interleaved (re, im): complex128 = 2 doubles,
 *     complex64 = 2 floats.
 *   - Argument errors return MATVIS_EINVAL synchronously and leave the context
 *     usable; HIP failures return MATVIS_EHIP; data errors found on the device
 *     (negative or non-finite flux, non-finite antenna positions) are reported
 *     by matvis_finish as MATVIS_EDATA (the visibilities are then undefined).
 *     No entry point aborts, exits or throws.  matvis_last_error gives text.
 *   - A context is used by one host thread at a time.
 */
#ifndef MATVIS_H
#define MATVIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct matvis_ctx matvis_ctx;

typedef enum {
    MATVIS_OK = 0,
    MATVIS_EINVAL = -1,       /* bad argument or shape */
    MATVIS_ENOMEM = -2,       /* device allocation failed */
    MATVIS_EHIP = -3,         /* a HIP runtime call failed */
    MATVIS_EUNSUPPORTED = -4, /* valid but unsupported combination */
    MATVIS_ESTATE = -5,       /* call not valid in the context's state */
    MATVIS_EDATA = -6         /* invalid input values detected on the device */
} matvis_status;

/* Arithmetic of step (v), V = Z Z^H.
 *   FP64  : complex128 beams, Z, products and output;
 *   FP32  : complex64 beams and Z, FP32 MFMA products accumulated in FP32
 *           over bounded source chunks, chunks combined in FP64, complex64 out;
 *   BF16X3: Z in FP32 split into bf16 hi + lo parts, V ~ hi hi^T + hi lo^T +
 *           lo hi^T on bf16 MFMA with FP32 accumulation, complex64 out.
 * In every mode the rotation and the phase range reduction are FP64. */
typedef enum { MATVIS_FP64 = 0, MATVIS_FP32 = 1, MATVIS_BF16X3 = 2 } matvis_precision;

/* Step (ii): beam evaluation at the visible sources. */
typedef enum {
    MATVIS_BEAM_BILINEAR = 0,  /* bilinear on the az/za grid */
    MATVIS_BEAM_BICUBIC = 1,   /* Keys cubic convolution (a = -1/2), Keys' end rows in za */
    MATVIS_BEAM_SURROGATE = 2  /* learned Fourier-feature network (see matvis_set_surrogate) */
} matvis_beam_mode;

/* Problem geometry and capacities, fixed for the context's lifetime.
 * Beam grid geometry: za_j = j * dza_rad for j < n_za (the last row is the
 * horizon, (n_za - 1) * dza_rad = pi/2); az_k = k * daz_rad, periodic with
 * n_az * daz_rad = 2 pi; az is measured from North through East. */
typedef struct {
    int32_t n_ant;        /* antennas (Sec. 3.5 input D) */
    int32_t n_feed;       /* feeds per antenna, 1 or 2 (Sec. 3.1) */
    int32_t n_ax;         /* E-field axes, 1 or 2 (Sec. 3.1) */
    int32_t n_beam;       /* unique beams (Sec. 3.5 inputs A and a_i) */
    int64_t max_src;      /* largest n_src a simulate call may pass */
    int32_t max_time;     /* largest n_time */
    int32_t max_freq;     /* largest n_freq */
    double latitude_rad;  /* l in Eq. (rotation) */
    int32_t precision;    /* matvis_precision */
    int32_t beam_mode;    /* matvis_beam_mode */
    int32_t n_za, n_az;   /* beam grid size (ignored for the surrogate) */
    double dza_rad, daz_rad;
    int64_t src_chunk;    /* sources per chunk (Sec. 6.4 chunking); 0 = automatic */
    int32_t batch_time;   /* times per device batch; 0 = automatic */
    int32_t batch_freq;   /* frequencies per device batch; 0 = automatic */
    int32_t flags;        /* MATVIS_FLAG_* bits */
    int64_t ksplit;       /* Z columns summed by one product work item before its partial
                             is stored (a multiple of 64); 0 = automatic.  FP32
                             accumulators see ksplit / 2 sequential updates, so this
                             bounds their rounding; the partials are summed in FP64. */
    int32_t tile;         /* product kernel variant, 0 = the library's choice.  Bits 0-3:
                             Z rows per 16-source stage formed by the multiply-first
                             waves, in units of 32 antennas (2, 3 or 4; 3 by default),
                             on the paths that split forming between two wave kinds
                             (MATVIS_PATH_SOURCES diagonal blocks: 2 or 3;
                             MATVIS_PATH_FUSED_BLOCKS: 2, 3 or 4).  Bit 4: the kernel
                             of the off-diagonal antenna-block pairs on
                             MATVIS_PATH_SOURCES with BF16X3: 0 puts each source's
                             coherency weight on the rows only (the plain fringe rows
                             of the other block as columns), 1 splits it as square
                             roots over both sides (FP32 always uses the latter).
                             Bit 6: 16 sources per stage instead of 32 on
                             MATVIS_PATH_FUSED_BLOCKS with BF16X3.
                             Bits 0-3 and 6 only reschedule work; bit 4 changes
                             the rounding (not the tolerance). */
} matvis_config;

#define MATVIS_FLAG_NO_GRAPH 1 /* launch kernels directly instead of replaying a captured hipGraph */
#define MATVIS_FLAG_UNFUSED 2  /* FP32 / BF16X3: write Z to device memory in a separate step
                                  (Alg. 2 step (iv)) instead of forming it inside the product */
#define MATVIS_FLAG_POLARISED_SKY 4 /* src_flux holds all four Stokes parameters per source and
                                       channel: the brightness matrix of Sec. 2.1,
                                       C = [[I + Q, U + iV], [U - iV, I - Q]] over the beam's two
                                       E-field axes, enters Eq. (matvistensorprod) through
                                       Z = A F M with M M^H = C (Eq. fullz; M is the lower
                                       Cholesky factor).  Needs n_ax = 2. */

/* Create a context on the current HIP device and allocate all scratch for the
 * capacities in *cfg.  Returns MATVIS_EINVAL for inconsistent sizes (n_feed or
 * n_ax not in {1, 2}, non-positive counts, grid smaller than 3 x 3 or whose
 * spacing does not span 0..pi/2 and 0..2 pi), MATVIS_ENOMEM if the device
 * cannot hold the scratch.  *out is NULL on failure. */
matvis_status matvis_init(const matvis_config *cfg, matvis_ctx **out);

/* Simulate every (t, f) instance, Alg. 2 steps (i)-(v).
 *   antpos    [n_ant][3] double, ENU metres (Sec. 3.5 input D).  Only
 *             differences matter; the library centres them on their mean.
 *   beam_idx  [n_ant] int32 in [0, n_beam) or NULL (all 0)  (input a_i).
 *   freqs     [n_freq] double, Hz, n_freq <= max_freq.
 *   lsts      [n_time] double, local sidereal time in radians; R(t) of
 *             Eq. (rotation) is built on the device with hour angle H = -LST.
 *   src_radec [2][n_src] double: row 0 right ascension, row 1 declination
 *             (Eq. xeq is evaluated on the device).  n_src <= max_src.
 *   src_flux  [n_freq][n_src] double, Stokes I per channel, >= 0 (input I);
 *             with MATVIS_FLAG_POLARISED_SKY [4][n_freq][n_src]: I, Q, U, V per
 *             channel, physical (I >= sqrt(Q^2 + U^2 + V^2), checked on the
 *             device to a relative 1e-9 and reported as MATVIS_EDATA).
 *   beam_grid [n_beam][n_freq][n_feed][n_ax][n_za][n_az] complex, complex128
 *             when precision is FP64 else complex64; NULL for the surrogate.
 *   vis       [n_time][n_freq][n_ant][n_ant][n_feed][n_feed] complex,
 *             complex128 for FP64 else complex64, fully written:
 *             vis[t][f][a][b][p][q] = sum_n sum_k Z[(a,p),(n,k)] conj(Z[(b,q),(n,k)]),
 *             exactly Hermitian (vis[b][a][q][p] = conj vis[a][b][p][q]).
 *   stream    hipStream_t as void*.
 * The call is asynchronous: it enqueues work on `stream` and returns. */
matvis_status matvis_simulate(matvis_ctx *ctx, const double *antpos, const int32_t *beam_idx, const double *freqs,
                              int32_t n_freq, const double *lsts, int32_t n_time, const double *src_radec,
                              int64_t n_src, const double *src_flux, const void *beam_grid, void *vis, void *stream);

/* ---- Redundancy-aware product (App. A) ----------------------------------
 * For arrays with many redundant baselines, only one representative pair per
 * redundant group is needed.  V'_x = A_x B_x^H (Eq. Vpx) over a few
 * sub-matrices whose rows A_x (first antennas) and B_x (second antennas) are
 * chosen by the appendix's density heuristic covers every requested pair at a
 * fraction of the full product's size.
 *
 * matvis_redundant_groups (host only, no device work): baselines are the
 * pairs (i, j), i <= j, in lexicographic order, n_ant (n_ant + 1) / 2 of
 * them; two are redundant when their antennas carry the same beams
 * (beam_idx, NULL = all 0) and x_i - x_j agree to within tol_m metres in every
 * component.  group[p] is the group of pair p (pair order), rep_a / rep_b the
 * first pair of each group (capacity n_ant (n_ant + 1) / 2), *n_unique the
 * number of groups.  Host pointers.  MATVIS_EINVAL for NULL pointers,
 * n_ant outside [1, 8192], tol_m <= 0 or non-finite positions. */
matvis_status matvis_redundant_groups(const double *antpos, const int32_t *beam_idx, int32_t n_ant, double tol_m,
                                      int32_t *group, int32_t *rep_a, int32_t *rep_b, int32_t *n_unique);

/* The appendix's heuristic for n_sub sub-matrices over the pairs (pair_a[u],
 * pair_b[u]) (host only): alpha [n_ant] receives the first antennas ordered
 * by multiplicity (descending, ties by index; *n_alpha of them), sizes
 * [n_sub] the number of them in each sub-matrix and density [n_sub] each
 * sub-matrix's covered-pair density; *n_sub_out <= n_sub is the count used
 * (at most *n_alpha). */
matvis_status matvis_submatrix_plan(const int32_t *pair_a, const int32_t *pair_b, int32_t n_pair, int32_t n_ant,
                                    int32_t n_sub, int32_t *alpha, int32_t *sizes, double *density, int32_t *n_alpha,
                                    int32_t *n_sub_out);

/* Plan the sub-matrix product for the pairs (pair_a[u], pair_b[u]) (host
 * arrays, antennas in [0, n_ant); any pairs, usually the representatives of
 * matvis_redundant_groups) with n_sub sub-matrices, and upload the plan to
 * the context's device.  Any precision: with Z in device memory (FP64, or
 * MATVIS_FLAG_UNFUSED) the sub-matrix rows are gathered from it; otherwise
 * (FP32 / BF16X3) they are formed in the product's stages from the beam and
 * the fringe phase, as the full product forms Z.  Allocates the plan's
 * scratch (so call it outside graph capture); replaces an earlier plan.  *size_out (may be NULL) receives the total sub-matrix size
 * sum_x |A_x| |B_x| in antenna pairs. */
matvis_status matvis_set_pairs(matvis_ctx *ctx, const int32_t *pair_a, const int32_t *pair_b, int32_t n_pair,
                               int32_t n_sub, int64_t *size_out);

/* matvis_simulate for the planned pairs only: the same inputs, and
 *   vis_pairs [n_time][n_freq][n_pair][n_feed][n_feed] complex (complex128 on
 *             FP64, else complex64), vis_pairs[t][f][u][p][q] = V[(a_u,p),(b_u,q)]
 *             of matvis_simulate.
 * Steps (i)-(iv) as in matvis_simulate, then the sub-matrix product and a
 * fixed-order FP64 sum of its k-splits.  MATVIS_ESTATE without a plan. */
matvis_status matvis_simulate_pairs(matvis_ctx *ctx, const double *antpos, const int32_t *beam_idx,
                                    const double *freqs, int32_t n_freq, const double *lsts, int32_t n_time,
                                    const double *src_radec, int64_t n_src, const double *src_flux,
                                    const void *beam_grid, void *vis_pairs, void *stream);

/* Synchronise the last stream used and report deferred device-side errors:
 * MATVIS_EDATA for invalid input values, MATVIS_EHIP for asynchronous HIP
 * failures.  Clears the device error flags. */
matvis_status matvis_finish(matvis_ctx *ctx);

/* Text of the last error on this context (never NULL; "" when none).  Valid
 * until the next call on the context. */
const char *matvis_last_error(const matvis_ctx *ctx);

/* Name of a status code. */
const char *matvis_status_string(int32_t status);

/* Release the context and all its device memory (after synchronising). */
void matvis_destroy(matvis_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Learned beam: a Fourier-feature MLP standing in for Alg. 2 step (ii).
 *
 * The network maps normalised inputs x = (u, v, w) = (az / 2 pi,
 * za / (pi / 2), (nu - nu_min) / (nu_max - nu_min)) to the 2 x 2 complex
 * Jones matrix J[p][k] (8 reals o = 0..7: re, im of (0,0), (0,1), (1,0), (1,1)):
 *   phi = (sin 2 pi Bff (u, v), cos 2 pi Bff (u, v))   Bff [128][2], integer az
 *                                               column (features periodic in az)
 *   h1 = SiLU(W1 phi + b1), h2..h4 = SiLU(W h + b) (width 128),
 *   g = W5 h4 + b5 [64],  out_o = sum_{k<8} T_k(2 w - 1) g[8 o + k]
 * (T_k Chebyshev polynomials of the first kind): the direction enters through
 * the network, the frequency through a degree-7 series per output, so the
 * simulator evaluates the network once per source and time and sums the
 * series for every channel.
 * Parameters are one FP32 device vector of MATVIS_MLP_N_PARAMS floats in the
 * order Bff, W1, b1, W2, b2, W3, b3, W4, b4, W5, b5 (row-major weights
 * [out][in]).  The four hidden-layer products round both operands to bf16
 * and accumulate in FP32; features, biases, SiLU and the series are FP32;
 * the head (W5, b5) is FP32 in training and split hi / lo into three bf16
 * products in inference.  The Fourier matrix is fixed (its gradient is zero
 * and Adam leaves it).
 * All arrays are device arrays; scalars and loss histories are host values.
 * ------------------------------------------------------------------------- */
#define MATVIS_MLP_N_PARAMS 90944

/* out [n][8] = network(x [n][3]), each row at its own w.  Allocates a bf16 copy of the weights.
 * params and out must be 16-byte aligned (MATVIS_EINVAL otherwise). */
matvis_status matvis_mlp_forward(const float *params, const float *x, int64_t n, float *out, void *stream);

/* Mean squared error L = sum (out - y)^2 / (8 n) and its gradient with respect
 * to every parameter (grad [MATVIS_MLP_N_PARAMS], loss [1], device).
 * fp32_math != 0 keeps the products in FP32 (a check mode).  Allocates
 * activation workspace for n rows. */
matvis_status matvis_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t n, int32_t fp32_math,
                                   float *grad, float *loss, void *stream);

/* matvis_mlp_loss_grad without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight training loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as
 * matvis_mlp_loss_grad, but the activation workspace is a fixed array of the
 * library's (34 MB of device memory, held on every GPU the library runs on
 * until the process ends), so n is limited to 4096 rows: larger n returns
 * MATVIS_EINVAL with a message on stderr.  No hipMalloc, hipFree or memset
 * node is issued.  Asynchronous on `stream` (it does not synchronise).
 * Every call on one GPU shares that GPU's workspace: calls that overlap in
 * time on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  The first call on each device looks up the
 * workspace's device address, so make it outside graph capture. */
matvis_status matvis_mlp_loss_grad_noalloc(const float *params, const float *x, const float *y, int64_t n,
                                           int32_t fp32_math, float *grad, float *loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on
 * params with first / second moment vectors m1, m2 of the same length. */
matvis_status matvis_mlp_adam(float *params, const float *grad, float *m1, float *m2, int64_t step, float lr,
                              void *stream);

/* Training pairs from the method's own interpolant (Sec. 3.4): out [n][8] =
 * beam of channel chan[i] at (za[i], az[i]) from a complex64 grid
 * [n_chan][n_feed][n_ax][n_za][n_az] (geometry as in matvis_config),
 * bilinear (bicubic = 0) or Keys bicubic (bicubic = 1); components beyond
 * n_feed x n_ax are 0.  If x is not NULL it receives the network inputs
 * x [n][3] = (az / 2 pi, za / (pi / 2), (chan_freq_hz[chan] - nu_min_hz) /
 * (nu_max_hz - nu_min_hz)), formed as matvis_simulate forms them.  chan is
 * checked on the host (MATVIS_EINVAL if outside [0, n_chan)); asynchronous
 * after that check. */
matvis_status matvis_beam_samples(const void *grid, int32_t n_chan, int32_t n_feed, int32_t n_ax, int32_t n_za,
                                  int32_t n_az, double dza_rad, double daz_rad, int32_t bicubic, const double *za,
                                  const double *az, const int32_t *chan, int64_t n, float *out,
                                  const double *chan_freq_hz, double nu_min_hz, double nu_max_hz, float *x,
                                  void *stream);

/* Train params in place on samples (x [n][3], y [n][8]) with Adam, mini-batches
 * of `batch` rows in an order reshuffled every epoch (seeded), learning rate
 * decaying geometrically from lr0 to lr1 over the epochs.  loss_history (host,
 * may be NULL) receives the mean batch loss of each epoch.  Synchronous;
 * allocates its workspace. */
matvis_status matvis_train_surrogate(float *params, const float *x, const float *y, int64_t n, int32_t batch,
                                     int32_t epochs, float lr0, float lr1, uint64_t seed, int32_t fp32_math,
                                     float *loss_history, void *stream);

/* Give a context created with beam_mode MATVIS_BEAM_SURROGATE its networks
 * (copied): params holds n_beam parameter vectors back to back
 * ([n_beam][MATVIS_MLP_N_PARAMS], one network per unique beam, antenna a using
 * network beam_idx[a]) and the frequency range that normalises w.  The
 * context must have FP32 or BF16X3 precision; beam_grid is then ignored by
 * matvis_simulate (NULL is accepted). */
matvis_status matvis_set_surrogate(matvis_ctx *ctx, const float *params, double nu_min_hz, double nu_max_hz);

/* ---------------------------------------------------------------------------
 * Autotuner for the batched product (the grouped persistent launch of many
 * (t, nu) instances).  It times matvis_simulate on the caller's own inputs and
 * returns in *best a copy of *base with the fastest product kernel variant
 * (tile), ksplit, src_chunk, batch_time and MATVIS_FLAG_UNFUSED choice, and
 * the time of one call in *best_ms (host pointers).  The search is coordinate
 * descent from the library's defaults over, in order: the block-pair kernel
 * (tile bit 4), the forming split (tile bits 0-3), the stage depth (tile bit 6), ksplit
 * (the path's default, two and
 * four times it, half and a quarter of it: the larger ones write fewer partial
 * sums and accumulate more terms in FP32, whose rounding grows about as the
 * square root of the split), src_chunk (default, 2^18, 2^20
 * sources), batch_time (default, 1, 2, 4, 8) and fused / unfused Z.  0, the
 * library's own choice, is a candidate on every axis, so the result is never
 * slower than the defaults as timed.  Candidates that do not fit in device
 * memory are skipped.  With beam_mode MATVIS_BEAM_SURROGATE, surrogate_params
 * ([n_beam][MATVIS_MLP_N_PARAMS], device) and nu_min_hz / nu_max_hz are given
 * to every candidate context as matvis_set_surrogate would (MATVIS_EINVAL if
 * surrogate_params is NULL); otherwise they are ignored.  If cache_path is
 * not NULL, results are read from and written to that JSON file, keyed by
 * GPU architecture, product path, rows, axes, unique beams, the polarised-sky
 * flag, the source count as a power-of-two bucket, times, channels,
 * precision and beam mode; a cached entry is returned without timing.  vis is
 * overwritten.  Synchronous.
 * ------------------------------------------------------------------------- */
matvis_status matvis_autotune(const matvis_config *base, const double *antpos, const int32_t *beam_idx,
                              const double *freqs, int32_t n_freq, const double *lsts, int32_t n_time,
                              const double *src_radec, int64_t n_src, const double *src_flux,
                              const void *beam_grid, void *vis, void *stream, const char *cache_path,
                              matvis_config *best, double *best_ms, const float *surrogate_params,
                              double nu_min_hz, double nu_max_hz);

/* ---------------------------------------------------------------------------
 * Per-step timing (the paper times each step of Alg. 2 separately, Sec. 6.1).
 * While enabled, matvis_simulate launches its kernels directly (no graph) and
 * brackets every launch of each step with a pair of HIP events on the
 * caller's stream.  matvis_profile_read synchronises those events, writes the
 * summed device time in milliseconds and the number of launches per step, in
 * the order of enum matvis_step, and forgets them.  ms and launches are HOST
 * arrays of MATVIS_N_STEPS entries.
 * ------------------------------------------------------------------------- */
typedef enum {
    MATVIS_STEP_SKY = 0,    /* rotation + compaction (count, scan, scatter) */
    MATVIS_STEP_BEAM = 1,   /* beam interpolation */
    MATVIS_STEP_ZFORM = 2,  /* phase + Z formation */
    MATVIS_STEP_HERK = 3,   /* the Z Z^H product kernel alone */
    MATVIS_STEP_REDUCE = 4, /* k-split reduction + Hermitian fill */
    MATVIS_STEP_OTHER = 5,  /* input preparation and the work-list prefix */
    MATVIS_STEP_HERK_PAIRS = 6, /* the product's second launch, where it has one: the
                                   off-diagonal antenna-block pairs (paths SOURCES and
                                   FUSED); the product's time is HERK + HERK_PAIRS */
    MATVIS_N_STEPS = 7
} matvis_step;

matvis_status matvis_profile_enable(matvis_ctx *ctx, int32_t enable);
matvis_status matvis_profile_read(matvis_ctx *ctx, double *ms, int64_t *launches);

/* Which kernel forms the product of Eq. zz for this context (fixed at init):
 *   MATVIS_PATH_Z_IN_HBM   Z is written to device memory by its own step and
 *                          V = Z Z^H reads it (FP64, or MATVIS_FLAG_UNFUSED);
 *   MATVIS_PATH_FUSED      Z formed in LDS per 128-row super-tile pair;
 *   MATVIS_PATH_FUSED_ROWS Z formed once per (instance, k-split) for all of
 *                          129..256 rows (BF16X3);
 *   MATVIS_PATH_SOURCES    2 feeds x 2 axes with one shared beam, more than
 *                          64 antennas (BF16X3 or FP32; blocks of 128
 *                          antennas, one item per block and two per block
 *                          pair): the axis sum is taken per source
 *                          first, V[(a,p),(b,q)] = sum_m F_a conj(F_b) C_pq(m),
 *                          so the product runs over sources, not over the
 *                          (source, axis) columns of Z -- half the
 *                          multiply-adds for the same V;
 *   MATVIS_PATH_FUSED_BLOCKS one feed, one axis, one shared beam, 257..384
 *                          antennas (BF16X3 or FP32): three items per
 *                          (instance, k-split), each a diagonal triangle with
 *                          the off-diagonal block that shares its rows, so
 *                          every row block is formed twice instead of three
 *                          or four times.
 * Returns the path, or a negative status for a NULL context. */
typedef enum {
    MATVIS_PATH_Z_IN_HBM = 0,
    MATVIS_PATH_FUSED = 1,
    MATVIS_PATH_FUSED_ROWS = 2,
    MATVIS_PATH_SOURCES = 3,
    MATVIS_PATH_FUSED_BLOCKS = 4
} matvis_product_path;

int32_t matvis_product_path_of(const matvis_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Step entry points: one hot-path step on caller buffers, using the context's
 * geometry and precision.  They exist so each kernel can be checked on its
 * own; matvis_simulate runs the same kernels.
 * ------------------------------------------------------------------------- */

/* Alg. 2 step (i) for n_time LSTs and n_src sources (n_time <= max_time,
 * n_src <= max_src):
 *   idx     [n_time][n_src] int32: ascending indices of sources with U > 0
 *           (first count[t] entries of row t are defined);
 *   count   [n_time] int32: visible sources per time;
 *   s_hat   [n_time][3][n_src] double: (E, N, U) of the visible sources, in
 *           the order of idx (may be NULL);
 *   za_az   [n_time][2][n_src] double: zenith angle and azimuth of the
 *           visible sources (may be NULL). */
matvis_status matvis_step_sky(matvis_ctx *ctx, const double *lsts, int32_t n_time, const double *src_radec,
                              int64_t n_src, int32_t *idx, int32_t *count, double *s_hat, double *za_az,
                              void *stream);

/* Alg. 2 step (ii) alone: beam values at n points given by zenith angle and
 * azimuth za_az [2][n] (double), from one channel's grid slice
 * grid [n_beam][n_feed][n_ax][n_za][n_az] (complex128 for FP64, else
 * complex64), with the context's beam mode (bilinear or bicubic).
 * Output A [n_beam][n_feed][n_ax][n] complex of the same width. */
matvis_status matvis_step_interp(matvis_ctx *ctx, const double *za_az, int64_t n, const void *grid, void *A,
                                 void *stream);

/* Step (v) alone: V = Z Z^H for an [n_row][n_col] complex matrix Z with
 * row stride ld elements (complex128 for FP64, else complex64), n_row <=
 * n_ant * n_feed, n_col <= n_ax * max_src.  Output V [n_row][n_row] of the
 * same complex width, fully written and Hermitian.  BF16X3 splits Z on the
 * device before the product. */
matvis_status matvis_step_herk(matvis_ctx *ctx, const void *Z, int32_t n_row, int64_t n_col, int64_t ld, void *V,
                               void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MATVIS_H */
