// Internal declarations shared by the HIP translation units of libmatvis.
// Everything here is gfx950 device code or host launch glue; the public
// boundary is include/matvis.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace mv {

constexpr double kSpeedOfLight = 299792458.0;  // m/s
constexpr int kColPad = 64;                    // Z columns are padded to a multiple of this (complex elements)
constexpr int kWave = 64;                      // CDNA wavefront width

enum Prec : int { P64 = 0, P32 = 1, PB3 = 2 };
enum Interp : int { BILINEAR = 0, BICUBIC = 1 };

// Device error flag bits (OR-ed into ctx->d_flags).
enum : int { FLAG_BAD_FLUX = 1, FLAG_BAD_ANTPOS = 2, FLAG_BAD_BEAM_IDX = 4 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Everything one batch of (t, f) instances needs to locate its data.
// Instance i of the batch is (t, f) = (t0 + i / nfb, f0 + i % nfb); its sky
// lives in time slot i / nfb of the sky buffers.
struct Batch {
    int32_t t0, f0, ntb, nfb;  // first time / frequency, and how many of each
    int32_t n_inst;            // ntb * nfb
};

// Lower-triangular square root M (M M^H = C) of a source's brightness matrix
// C = [[I + Q, U + iV], [U - iV, I - Q]] (Sec. 2.1): the Cholesky factor
//   M = [[sqrt(I + Q), 0], [(U - iV) / sqrt(I + Q), sqrt(I - Q - (U^2 + V^2) / (I + Q))]],
// and M = [[0, 0], [0, sqrt(I - Q)]] when I + Q = 0.  Unlike the closed form of
// App. B (which divides by U - iV and by T) it exists for every physical source,
// unpolarised and fully polarised ones included; an unpolarised source gives
// M = sqrt(I) 1 exactly.  Rounding below zero under the last root is clamped.
struct PolSqrt {
    double m00, m10x, m10y, m11;
};
__device__ inline PolSqrt pol_sqrt(double si, double sq, double su, double sv) {
    PolSqrt r;
    const double c00 = si + sq;
    if (c00 > 0.0) {
        r.m00 = sqrt(c00);
        r.m10x = su / r.m00;
        r.m10y = -sv / r.m00;
        const double d = (si - sq) - (su * su + sv * sv) / c00;
        r.m11 = d > 0.0 ? sqrt(d) : 0.0;
    } else {
        r.m00 = r.m10x = r.m10y = 0.0;
        const double d = si - sq;
        r.m11 = d > 0.0 ? sqrt(d) : 0.0;
    }
    return r;
}
// One feed's row of A M (Eq. fullz): (a0, a1) = A[p][0], A[p][1] -> (A M)[p][0], (A M)[p][1].
template <typename R>
__device__ inline void apply_pol_sqrt(const PolSqrt &m, R a0x, R a0y, R a1x, R a1y, R &o0x, R &o0y, R &o1x, R &o1y) {
    const R m00 = (R)m.m00, m10x = (R)m.m10x, m10y = (R)m.m10y, m11 = (R)m.m11;
    o0x = a0x * m00 + (a1x * m10x - a1y * m10y);
    o0y = a0y * m00 + (a1x * m10y + a1y * m10x);
    o1x = a1x * m11;
    o1y = a1y * m11;
}

// Device-side sky buffers of one time batch and one source chunk.
struct SkyBufs {
    const double *xeq;  // [3][ld_xeq] unit vectors, Eq. (xeq)
    int64_t ld_xeq;
    const double *rot;  // [max_time][9] rotation matrices, Eq. (rotation)
    int32_t *blk_count; // [ntb][nblk]
    int32_t *blk_off;   // [ntb][nblk]
    int32_t *count;     // [ntb] visible sources in the chunk
    int32_t *idx;       // [ntb][ld_src] absolute source indices, ascending
    double *s_hat;      // [ntb][3][ld_src] (E, N, U)
    double *za_az;      // [ntb][2][ld_src]
    int64_t ld_src;     // row stride of the per-time arrays (>= chunk size)
    const int32_t *perm; // [n_src] original number of the source at each sky position, or null
};

// ---- sky (kernels_sky.hip) -------------------------------------------------
hipError_t launch_xeq(const double *radec, int64_t n_src, double *xeq, int64_t ld, hipStream_t s);
// Eq. (xeq) with the sources put in sky-cell order (stable): xeq[.][pos] is
// source perm[pos].  Scratch: xeq_in [3][ld] doubles, cell [ld] int16, hist
// [sort_hist_entries(ld)] int32.
struct SortBufs {
    double *xeq_in;
    int16_t *cell;
    int32_t *hist;
    int32_t *perm;
};
hipError_t launch_xeq_sorted(const double *radec, int64_t n_src, int64_t ld, SortBufs sb, double *xeq, hipStream_t s);
int64_t sort_hist_entries(int64_t max_src);
hipError_t launch_rotmats(const double *lsts, int32_t n_time, double latitude, double *rot, hipStream_t s);
// n_flux values of Stokes I are checked (>= 0, finite); with pol the four planes
// [4][n_flux] are checked for a physical brightness matrix.
hipError_t launch_prep_inputs(const double *antpos, int32_t n_ant, const int32_t *beam_idx, int32_t n_beam,
                              const double *flux, int64_t n_flux, int pol, double *antc, int32_t *bidx,
                              int32_t *flags, hipStream_t s);
hipError_t launch_sky(const SkyBufs &b, int32_t t0, int32_t ntb, int64_t c0, int64_t nsrc_chunk, hipStream_t s);

// ---- beam (kernels_beam.hip) -----------------------------------------------
struct InterpArgs {
    const void *grid;        // [n_beam][n_freq_grid][n_feed][n_ax][n_za][n_az]
    int32_t n_freq_grid;     // channels in the grid array
    int32_t n_beam, n_feed, n_ax, n_za, n_az;
    double dza, daz;
    const double *za_az;     // [nslots][2][ld_src]
    const int32_t *count;    // [nslots] visible counts, or null -> fixed_count
    int64_t fixed_count;
    int64_t ld_src;
    void *A;                 // [n_inst][n_beam][n_feed][n_ax][ld_src]
    int64_t max_m;           // grid size along sources
    // optional: multiply by sqrt(I) of the source (B = sqrt(I) A for the fused product)
    const int32_t *idx;      // [nslots][ld_src] absolute source indices, or null
    const double *flux;      // [n_freq][n_src], or the Stokes planes [4][n_freq][n_src] when pol
    int64_t n_src;
    // polarised sky: B = A M with M of pol_sqrt (needs n_ax = 2 and idx set);
    // Stokes plane s starts at flux + s * stokes_stride
    int32_t pol;
    int64_t stokes_stride;
    // launch_interp_tf only, optional: scratch for each (slot, source)'s stencil,
    // interp_stencil_bytes(prec, ld_src, nslots) bytes; null -> formed in the kernel
    void *stencil;
};
hipError_t launch_interp(int prec, int mode, const InterpArgs &a, const Batch &bt, hipStream_t s);
// stencil scratch of launch_interp_tf: the packed (first row, first column) and
// the 4 row and 4 column weights of every (slot, source), in the precision's real type
inline size_t interp_stencil_bytes(int prec, int64_t ld_src, int nslots) {
    return (size_t)nslots * ld_src * (4 + 8 * (prec == P64 ? 8 : 4));
}
// Channel-interleaved copy of the beam grids, T[b][za][az][f][c] (c = feed * n_ax + axis),
// so one grid point's channels and components are one contiguous run; runs are
// (n_freq * ncomp) rounded up to even long, and the buffer needs
// grid_interleave_elems(...) complex values (4 of slack at the end).
hipError_t launch_grid_interleave(int prec, const void *grid, int n_beam, int n_freq, int ncomp, int n_za, int n_az,
                                  void *T, hipStream_t s);
inline int64_t grid_interleave_elems(int n_beam, int n_freq, int ncomp, int n_za, int n_az) {
    return (int64_t)n_beam * n_za * n_az * ((n_freq * ncomp + 1) & ~1) + 4;
}
// The beam step on the interleaved grid: a.grid = T with a.n_freq_grid channels;
// a group of lanes per (visible source, time slot, group of 4 channels of the
// batch).  With a.stencil set, each (slot, source)'s stencil is formed once by
// a pass of its own instead of by every lane of every group.  Needs n_za >= 4
// and n_za, n_az < 65536.
hipError_t launch_interp_tf(int prec, int mode, const InterpArgs &a, const Batch &bt, hipStream_t s);

// ---- Z formation (kernels_z.hip) -------------------------------------------
struct ZformArgs {
    const double *antc;      // [n_ant][3] centred ENU
    const int32_t *bidx;     // [n_ant] sanitised beam index
    const double *freqs;     // [n_freq]
    const double *flux;      // [n_freq][n_src], or null when A already carries the sky (B = sqrt(I) A or A M)
    int64_t n_src;
    const int32_t *idx;      // [nslots][ld_src]
    const double *s_hat;     // [nslots][3][ld_src]
    const int32_t *count;    // [nslots]
    const void *A;           // [n_inst][n_beam][n_feed][n_ax][ld_src]
    int64_t ld_src;
    int32_t n_ant, n_feed, n_ax, n_beam;
    void *Z;                 // FP64/FP32: [n_inst][n_rows_pad][ldz] complex; BF16X3: hi plane
    void *Z_lo;              // BF16X3 lo plane, same shape (4 B per complex)
    int64_t ldz;             // complex elements per row
    int32_t n_rows_pad;
    int64_t max_m;           // launch size along sources (>= padded count)
};
hipError_t launch_zform(int prec, const ZformArgs &a, const Batch &bt, hipStream_t s);
// Copy a caller's dense Z [n_row][ld] into the padded scratch layout (splitting
// for BF16X3); rows n_row..n_rows_pad-1 and columns n_col..n_col_pad-1 become zero.
hipError_t launch_z_import(int prec, const void *Zin, int32_t n_row, int32_t n_rows_pad, int64_t n_col, int64_t ld,
                           void *Z, void *Z_lo, int64_t ldz, int64_t n_col_pad, hipStream_t s);

// ---- HERK (kernels_herk.hip) -----------------------------------------------
struct HerkArgs {
    const void *Z;           // as in ZformArgs
    const void *Z_lo;
    int64_t ldz;
    int64_t inst_stride;     // elements between instances in Z
    int32_t n_rows;          // N = n_ant * n_feed
    int32_t n_rows_pad;      // multiple of the super-tile size
    const int32_t *count;    // [nslots] visible counts (K = n_ax * count), or null -> fixed_k
    int64_t fixed_k;
    int32_t n_ax;
    int32_t nfb;             // instance i uses count slot i / nfb
    int32_t n_inst;
    int64_t ksplit;          // complex columns per work item (multiple of 64)
    int32_t max_splits;      // partial slots per instance
    void *part;              // [n_inst][max_splits][n_rows_pad][n_rows_pad] complex partials
    int32_t *work;           // [n_inst + 1] item prefix
    int32_t *nsplit;         // [n_inst] k-splits of each instance (built with work)
    int32_t *kcols;          // [n_inst] columns per k-split of each instance (a multiple of 64)
    int32_t balance_grid;    // > 0: add k-splits so the items fill whole waves of this many workgroups
    int32_t grid;            // persistent grid size (multiple of 8)
};
int herk_super_tile(int prec);
int herk_occupancy(int prec);  // resident workgroups per CU
// Item prefix over the batch (k_worklist), then the persistent product kernel.
// unit != 0 counts k-splits only (the fused product multiplies by its item kinds).
// Instance i gets nsplit[i] k-splits of kcols[i] <= ksplit columns (the last
// one partial); without balancing that is ceil(K_i / ksplit) of ksplit.
hipError_t launch_worklist(int prec, const HerkArgs &a, int unit, hipStream_t s);
hipError_t launch_herk(int prec, const HerkArgs &a, hipStream_t s);

// Product with Z formed in LDS (kernels_herk_fused.hip); FP32 and BF16X3 only.
struct FusedArgs {
    const double *antc;      // [n_ant][3] centred ENU
    const int32_t *bidx;     // [n_ant]
    const double *freqs;     // [n_freq]
    const double *s_hat;     // [nslots][3][ld_src]
    const void *B;           // sqrt(I) A, complex64 [n_inst][n_beam][n_feed][n_ax][ld_src]
    const int32_t *count;    // [nslots]
    int64_t ld_src;
    int32_t n_ant, n_feed, n_ax, n_beam;
    int32_t n_rows_pad;
    int32_t f0, nfb, n_inst;
    const int32_t *kcols;    // [n_inst] columns per k-split (launch_worklist)
    int32_t max_splits;
    void *part;
    int32_t *work;           // built by launch_worklist
    int32_t grid;
    int32_t tile;            // kernel variant (matvis_config.tile): bits 0-3 the forming split
};
// which: FUSED_ALL every launch of the path; FUSED_FIRST its first launch only (the
// diagonal blocks, or the only launch); FUSED_PAIRS its second launch only (the
// off-diagonal block pairs of paths SOURCES and FUSED; nothing on the others).
enum { FUSED_ALL = 0, FUSED_FIRST = 1, FUSED_PAIRS = 2 };
hipError_t launch_herk_fused(int prec, const FusedArgs &a, hipStream_t s, int which = FUSED_ALL);
// whether the path of these arguments has a second (block-pair) launch
bool fused_has_pairs(int prec, const FusedArgs &a);
int herk_fused_occupancy(int prec);
// the library's k-split for a precision and product path (matvis_config.ksplit = 0)
int64_t default_ksplit(int prec, bool over_sources, bool three_blocks);
// product kernel launch_herk_fused picks (a matvis_product_path value, never Z_IN_HBM)
int fused_path(int prec, int n_feed, int n_ax, int n_beam, int n_ant, int n_rows_pad);

// Redundancy-aware sub-matrix product (App. A, Eq. Vpx) on Z in device memory,
// FP64, FP32 and BF16X3 (kernels_herk.hip).  Tiles are kSubmatTile square: small, because
// sub-matrices are often thin (tens of rows against hundreds), and a tile's
// padding is computed for nothing.
constexpr int kSubmatTile = 32;
struct SubmatArgs {
    const void *Z;           // [n_inst][Np][ldz] as written by launch_zform (BF16X3: hi plane)
    const void *Z_lo;        // BF16X3 lo plane
    int64_t ldz;
    int64_t inst_stride;     // elements between instances
    const int32_t *rows;     // [n_tiles][2][ST]: the tile's A rows then B rows of Z, -1 = padding
    int32_t n_tiles;
    const int32_t *count;    // [nslots] visible counts (K = n_ax * count)
    int64_t fixed_k;
    int32_t n_ax, nfb, n_inst;
    int64_t ksplit;          // columns per k-split (multiple of 16)
    int32_t max_splits;
    void *part;              // [n_inst][max_splits][n_tiles][ST][ST] complex partials
    // Z formed in the stages instead of read (launch_submat_fused, FP32 / BF16X3):
    // Z[(a, p), (m, k)] = B[inst][beam(a)][p][k][m] F_a(m) from these inputs
    const double *antc;      // [n_ant][3] centred ENU
    const int32_t *bidx;     // [n_ant] sanitised beam index
    const double *freqs;     // [n_freq]
    const double *s_hat;     // [nslots][3][ld_src]
    const void *B;           // sqrt(I) A (or A M), complex64 [n_inst][n_beam][n_feed][n_ax][ld_src]
    int64_t ld_src;
    int32_t n_feed, n_beam, f0;
};
hipError_t launch_submat(int prec, const SubmatArgs &a, hipStream_t s);
hipError_t launch_submat_fused(int prec, const SubmatArgs &a, hipStream_t s);
struct SubmatReduceArgs {
    const void *part;
    int32_t n_tiles, max_splits, st;
    const int32_t *loc;      // [n_pair][n_feed][n_feed][2]: tile, r * ST + c
    int32_t n_pair, n_feed;
    const int32_t *count;
    int64_t fixed_k;
    int32_t n_ax, nfb, n_inst;
    int64_t ksplit;
    double *vacc;            // [n_inst][n_pair][n_feed][n_feed] complex128 running sums
    int32_t first, last;
    void *out;               // [n_time][n_freq][n_pair][n_feed][n_feed]
    int32_t n_freq_total;
    Batch bt;
};
hipError_t launch_submat_reduce(int prec, const SubmatReduceArgs &a, hipStream_t s);

// Host side (redundancy.hip): baseline redundancy groups and the App. A plan.
namespace red {
int64_t groups(const double *antpos, const int32_t *beam_idx, int n_ant, double tol, int32_t *group, int32_t *rep_a,
               int32_t *rep_b);
struct Plan {
    std::vector<int> alpha, sizes;           // ordered first antennas, sub-matrix sizes
    std::vector<std::vector<int>> A, B;      // antennas of A_x (alpha order), of B_x (ascending)
    std::vector<double> density;
};
Plan plan(const int32_t *pa, const int32_t *pb, int n_pair, int n_ant, int n_sub);
}  // namespace red

struct ReduceArgs {
    const void *part;
    int32_t n_rows, n_rows_pad, max_splits;
    const int32_t *count;
    int64_t fixed_k;
    int32_t n_ax, nfb, n_inst;
    int64_t ksplit;
    const int32_t *nsplit;   // [n_inst] k-splits per instance, or null: ceil(K / ksplit)
    double *vacc;            // [n_inst][n_rows][n_rows] complex128 running sums (multi-chunk)
    int32_t first, last;     // first chunk: assign; last chunk: write the output
    void *out;               // output base
    int32_t out_kind;        // 0: vis layout [t][f][a][b][p][q]; 1: plain [r][c]
    int32_t n_ant, n_feed, n_freq_total;
    Batch bt;
};
hipError_t launch_reduce(int prec, const ReduceArgs &a, hipStream_t s);

}  // namespace mv
