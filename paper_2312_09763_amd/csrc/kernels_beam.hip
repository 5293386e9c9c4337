// Alg. 2 step (ii): beam (Jones terms) at the visible sources' (za, az) on an
// az/za grid whose pole is the zenith (Sec. 3.4).
//
// Grid geometry: za_j = j dza for j < n_za (last row on the horizon),
// az_k = k daz, periodic in az.  Two interpolants, both defined in index space:
//   bilinear : za cell j0 = clamp(floor(za/dza), 0, n_za - 2);
//   bicubic  : Keys (1981) cubic convolution with a = -1/2 on a 4 x 4
//              stencil, periodic in az, and Keys' end conditions for the two
//              rows beyond the za ends: g[-1] = 3 g0 - 3 g1 + g2 and
//              g[n] = 3 g[n-1] - 3 g[n-2] + g[n-3].  Interpolation near the
//              zenith therefore runs along the source's own meridian, away
//              from the pole.
// One thread per (visible source, instance); the taps are read through the
// L2/MALL (a 0.5 deg polarised channel is 4.2 MB in complex64).  The Keys
// weights are evaluated in Horner form of the fraction.
#include "internal.h"

namespace mv {

namespace {

template <typename R>
struct CT;
template <>
struct CT<float> {
    typedef float2 T;
};
template <>
struct CT<double> {
    typedef double2 T;
};

// Keys weights for offsets -1, 0, 1, 2 at fraction t in [0, 1).
template <typename R>
__device__ inline void keys_weights(R t, R w[4]) {
    const R t2 = t * t, t3 = t2 * t;
    w[0] = R(-0.5) * t3 + t2 - R(0.5) * t;
    w[1] = R(1.5) * t3 - R(2.5) * t2 + R(1);
    w[2] = R(-1.5) * t3 + R(2) * t2 + R(0.5) * t;
    w[3] = R(0.5) * t3 - R(0.5) * t2;
}

template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_interp(InterpArgs a, Batch bt) {
    typedef typename CT<R>::T C;
    const int inst = blockIdx.y;
    const int slot = inst / bt.nfb;
    const int f = bt.f0 + inst % bt.nfb;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = a.count ? a.count[slot] : a.fixed_count;
    if (m >= M) return;
    const double za = a.za_az[(int64_t)slot * 2 * a.ld_src + m];
    const double az = a.za_az[(int64_t)slot * 2 * a.ld_src + a.ld_src + m];
    // cell and fractions: integer parts in FP64, fractions in the path's precision
    const double u = za / a.dza, v = az / a.daz;
    int j0 = (int)floor(u);
    j0 = j0 < 0 ? 0 : (j0 > a.n_za - 2 ? a.n_za - 2 : j0);
    const R t = (R)(u - j0);
    const double kf = floor(v);
    const R sfrac = (R)(v - kf);
    int k0 = (int)kf % a.n_az;
    if (k0 < 0) k0 += a.n_az;
    const int n_az = a.n_az;
    const int64_t plane = (int64_t)a.n_za * n_az;
    const int ncomp = a.n_feed * a.n_ax;
    const C *grid = (const C *)a.grid;
    C *out = (C *)a.A + (int64_t)inst * a.n_beam * ncomp * a.ld_src;
    // B = sqrt(I) A when the product forms Z itself
    const R sq = a.idx ? (R)sqrt(a.flux[(int64_t)f * a.n_src + a.idx[(int64_t)slot * a.ld_src + m]]) : R(1);

    if (MODE == BILINEAR) {
        const int k1 = k0 + 1 == n_az ? 0 : k0 + 1;
        const R w00 = (R(1) - t) * (R(1) - sfrac), w01 = (R(1) - t) * sfrac;
        const R w10 = t * (R(1) - sfrac), w11 = t * sfrac;
        for (int b = 0; b < a.n_beam; b++)
            for (int c = 0; c < ncomp; c++) {
                const C *g = grid + ((int64_t)(b * a.n_freq_grid + f) * ncomp + c) * plane;
                const C g00 = g[(int64_t)j0 * n_az + k0], g01 = g[(int64_t)j0 * n_az + k1];
                const C g10 = g[(int64_t)(j0 + 1) * n_az + k0], g11 = g[(int64_t)(j0 + 1) * n_az + k1];
                C r;
                r.x = sq * (w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x);
                r.y = sq * (w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y);
                out[((int64_t)b * ncomp + c) * a.ld_src + m] = r;
            }
    } else {
        R wj[4], wk[4];
        keys_weights<R>(t, wj);
        keys_weights<R>(sfrac, wk);
        int kc[4];
        for (int d = 0; d < 4; d++) {
            int k = k0 - 1 + d;
            kc[d] = k < 0 ? k + n_az : (k >= n_az ? k - n_az : k);
        }
        const int n_za = a.n_za;
        for (int b = 0; b < a.n_beam; b++)
            for (int c = 0; c < ncomp; c++) {
                const C *g = grid + ((int64_t)(b * a.n_freq_grid + f) * ncomp + c) * plane;
                R accx = 0, accy = 0;
                for (int dj = 0; dj < 4; dj++) {
                    const int j = j0 - 1 + dj;
                    R rx = 0, ry = 0;  // az-convolved row j
                    if (j >= 0 && j < n_za) {
                        const C *row = g + (int64_t)j * n_az;
                        for (int d = 0; d < 4; d++) {
                            const C v4 = row[kc[d]];
                            rx += wk[d] * v4.x;
                            ry += wk[d] * v4.y;
                        }
                    } else {
                        // Keys end row: 3 r0 - 3 r1 + r2 from the three rows nearest the end
                        const int e0 = j < 0 ? 0 : n_za - 1, step = j < 0 ? 1 : -1;
                        const R cf[3] = {R(3), R(-3), R(1)};
                        for (int q = 0; q < 3; q++) {
                            const C *row = g + (int64_t)(e0 + q * step) * n_az;
                            R qx = 0, qy = 0;
                            for (int d = 0; d < 4; d++) {
                                const C v4 = row[kc[d]];
                                qx += wk[d] * v4.x;
                                qy += wk[d] * v4.y;
                            }
                            rx += cf[q] * qx;
                            ry += cf[q] * qy;
                        }
                    }
                    accx += wj[dj] * rx;
                    accy += wj[dj] * ry;
                }
                C r;
                r.x = sq * accx;
                r.y = sq * accy;
                out[((int64_t)b * ncomp + c) * a.ld_src + m] = r;
            }
    }
}

}  // namespace

hipError_t launch_interp(int prec, int mode, const InterpArgs &a, const Batch &bt, hipStream_t s) {
    if (bt.n_inst <= 0 || a.max_m <= 0) return hipSuccess;
    dim3 g((unsigned)((a.max_m + 255) / 256), bt.n_inst);
    if (prec == P64) {
        if (mode == BILINEAR)
            k_interp<double, BILINEAR><<<g, 256, 0, s>>>(a, bt);
        else
            k_interp<double, BICUBIC><<<g, 256, 0, s>>>(a, bt);
    } else {
        if (mode == BILINEAR)
            k_interp<float, BILINEAR><<<g, 256, 0, s>>>(a, bt);
        else
            k_interp<float, BICUBIC><<<g, 256, 0, s>>>(a, bt);
    }
    return hipGetLastError();
}

}  // namespace mv
