// Alg. 2 steps (iii)-(iv): the per-antenna matrix of Eq. (littlez),
//   Z[(a, p)][(n, k)] = sqrt(I_n) A_{beam(a), p, k}(n) F_a(n),
//   F_a(n) = exp(-2 pi i nu x_a . s_n / c)      (fringe factorisation, Sec. 3.2).
//
// The phase is reduced in FP64 before any trigonometry: p = (nu/c) x_a . s_n
// in cycles, r = p - rint(p) in [-1/2, 1/2], then F = cospi(2r) - i sinpi(2r)
// (FP32 sincospi on the FP32 / BF16X3 paths, FP64 on the FP64 path).  The tau
// matrix of Alg. 2 step (iii) is never stored.
//
// Layout written: row-major [n_rows_pad][ldz] per instance, row r = a n_feed + p,
// column c = n n_ax + k, complex interleaved (complex128 on FP64, complex64 on
// FP32).  BF16X3 writes two planes of packed bf16 pairs (re low half, im high
// half): hi = bf16(z), lo = bf16(z - hi), both round-to-nearest-even.
// Columns past n_ax * count up to the next multiple of 64 are written as zero
// so the product kernel can step over whole 16-column chunks.
//
// One thread per visible source; each block loops over a group of antennas so
// the source's direction, flux and beam are loaded once and reused, and the
// stores of consecutive threads are contiguous.
#include "internal.h"

namespace mv {

namespace {

constexpr int kAntGroup = 16;

__device__ inline uint32_t bf16_bits_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline float bf16_bits_to_float(uint32_t h) { return __uint_as_float(h << 16); }

// Split a complex64 value into packed bf16 (hi, lo) words.
__device__ inline void split_bf16(float re, float im, uint32_t &hi, uint32_t &lo) {
    uint32_t hr = bf16_bits_rne(re), hi_ = bf16_bits_rne(im);
    uint32_t lr = bf16_bits_rne(re - bf16_bits_to_float(hr));
    uint32_t li = bf16_bits_rne(im - bf16_bits_to_float(hi_));
    hi = hr | (hi_ << 16);
    lo = lr | (li << 16);
}

template <int PREC>
__global__ void __launch_bounds__(256) k_zform(ZformArgs a, Batch bt) {
    typedef typename std::conditional<PREC == P64, double, float>::type R;
    typedef typename std::conditional<PREC == P64, double2, float2>::type C;
    const int inst = blockIdx.z;
    const int slot = inst / bt.nfb;
    const int f = bt.f0 + inst % bt.nfb;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = a.count[slot];
    const int nx = a.n_ax, nf = a.n_feed;
    const int64_t kpad = ((nx * M + kColPad - 1) / kColPad) * kColPad;
    const int64_t mpad = (kpad + nx - 1) / nx;
    if (m >= mpad) return;
    const int a0 = blockIdx.y * kAntGroup;
    const int a1 = a0 + kAntGroup < a.n_ant ? a0 + kAntGroup : a.n_ant;
    const bool live = m < M;
    const int64_t ld = a.ld_src;
    const int64_t zinst = (int64_t)inst * a.n_rows_pad * a.ldz;

    double sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
    if (live) {
        const double *sh = a.s_hat + (int64_t)slot * 3 * ld;
        sx = sh[m];
        sy = sh[ld + m];
        sz = sh[2 * ld + m];
        sq = 1.0;
        if (a.flux) {  // else the beam step already carries the sky (polarised: A M)
            const int32_t n = a.idx[(int64_t)slot * ld + m];
            sq = sqrt(a.flux[(int64_t)f * a.n_src + n]);
        }
    }
    const double nu_c = a.freqs[f] / kSpeedOfLight;
    const int ncomp = nf * nx;
    const C *Ab = (const C *)a.A + (int64_t)inst * a.n_beam * ncomp * ld;

    C w[4];  // sqrt(I) A for (p, k) of the current beam
    int cur_b = -1;
    for (int ant = a0; ant < a1; ant++) {
        C z[4];
        if (live) {
            const int b = a.bidx[ant];
            if (b != cur_b) {
                for (int c = 0; c < ncomp; c++) {
                    C v = Ab[((int64_t)b * ncomp + c) * ld + m];
                    w[c].x = (R)sq * v.x;
                    w[c].y = (R)sq * v.y;
                }
                cur_b = b;
            }
            const double *x = a.antc + 3 * ant;
            const double p = nu_c * (x[0] * sx + x[1] * sy + x[2] * sz);
            const double r = p - rint(p);
            R sn, cs;
            if constexpr (PREC == P64)
                sincospi(-2.0 * r, &sn, &cs);
            else
                sincospif(-2.0f * (float)r, &sn, &cs);
            for (int c = 0; c < ncomp; c++) {
                z[c].x = w[c].x * cs - w[c].y * sn;
                z[c].y = w[c].x * sn + w[c].y * cs;
            }
        } else {
            for (int c = 0; c < ncomp; c++) {
                z[c].x = 0;
                z[c].y = 0;
            }
        }
        for (int p = 0; p < nf; p++) {
            const int64_t row = (int64_t)ant * nf + p;
            const int64_t off = zinst + row * a.ldz + m * nx;
            if constexpr (PREC == PB3) {
                uint32_t *hi = (uint32_t *)a.Z + off;
                uint32_t *lo = (uint32_t *)a.Z_lo + off;
                if (nx == 2) {
                    uint32_t h0, l0, h1, l1;
                    split_bf16(z[p * 2].x, z[p * 2].y, h0, l0);
                    split_bf16(z[p * 2 + 1].x, z[p * 2 + 1].y, h1, l1);
                    *(uint2 *)hi = make_uint2(h0, h1);
                    *(uint2 *)lo = make_uint2(l0, l1);
                } else {
                    uint32_t h0, l0;
                    split_bf16(z[p].x, z[p].y, h0, l0);
                    *hi = h0;
                    *lo = l0;
                }
            } else {
                C *zp = (C *)a.Z + off;
                for (int k = 0; k < nx; k++) zp[k] = z[p * nx + k];
            }
        }
    }
}

template <int PREC>
__global__ void k_z_import(const void *Zin, int n_row, int64_t n_col, int64_t ld, void *Z, void *Z_lo, int64_t ldz,
                           int64_t n_col_pad) {
    typedef typename std::conditional<PREC == P64, double2, float2>::type C;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= n_col_pad) return;
    C v;
    v.x = 0;
    v.y = 0;
    if (r < n_row && c < n_col) v = ((const C *)Zin)[(int64_t)r * ld + c];
    const int64_t o = (int64_t)r * ldz + c;
    if constexpr (PREC == PB3) {
        uint32_t h, l;
        split_bf16((float)v.x, (float)v.y, h, l);
        ((uint32_t *)Z)[o] = h;
        ((uint32_t *)Z_lo)[o] = l;
    } else {
        ((C *)Z)[o] = v;
    }
}

}  // namespace

hipError_t launch_zform(int prec, const ZformArgs &a, const Batch &bt, hipStream_t s) {
    if (bt.n_inst <= 0 || a.max_m <= 0) return hipSuccess;
    dim3 g((unsigned)((a.max_m + 255) / 256), (a.n_ant + kAntGroup - 1) / kAntGroup, bt.n_inst);
    if (prec == P64)
        k_zform<P64><<<g, 256, 0, s>>>(a, bt);
    else if (prec == P32)
        k_zform<P32><<<g, 256, 0, s>>>(a, bt);
    else
        k_zform<PB3><<<g, 256, 0, s>>>(a, bt);
    return hipGetLastError();
}

hipError_t launch_z_import(int prec, const void *Zin, int32_t n_row, int32_t n_rows_pad, int64_t n_col, int64_t ld,
                           void *Z, void *Z_lo, int64_t ldz, int64_t n_col_pad, hipStream_t s) {
    if (n_rows_pad <= 0 || n_col_pad <= 0) return hipSuccess;
    dim3 g((unsigned)((n_col_pad + 255) / 256), n_rows_pad);
    if (prec == P64)
        k_z_import<P64><<<g, 256, 0, s>>>(Zin, n_row, n_col, ld, Z, Z_lo, ldz, n_col_pad);
    else if (prec == P32)
        k_z_import<P32><<<g, 256, 0, s>>>(Zin, n_row, n_col, ld, Z, Z_lo, ldz, n_col_pad);
    else
        k_z_import<PB3><<<g, 256, 0, s>>>(Zin, n_row, n_col, ld, Z, Z_lo, ldz, n_col_pad);
    return hipGetLastError();
}

}  // namespace mv
