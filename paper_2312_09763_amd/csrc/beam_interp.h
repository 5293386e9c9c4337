// Beam interpolation at one (za, az) point on the az/za grid with the zenith
// as pole (Sec. 3.4), shared by the beam step and the training-sample
// generator of the learned beam.
//
// Grid: za_j = j dza (j < n_za, last row on the horizon), az_k = k daz,
// periodic in az; both interpolants are defined in index space.
//   bilinear : za cell j0 = clamp(floor(za/dza), 0, n_za - 2);
//   bicubic  : Keys (1981) cubic convolution, a = -1/2, 4 x 4 stencil,
//              periodic in az, with Keys' end rows g[-1] = 3 g0 - 3 g1 + g2 and
//              g[n] = 3 g[n-1] - 3 g[n-2] + g[n-3], so near the zenith the
//              stencil runs along the point's meridian, away from the pole.
#pragma once

#include "internal.h"

namespace mv {

template <typename R>
struct CplxOf;
template <>
struct CplxOf<float> {
    typedef float2 T;
};
template <>
struct CplxOf<double> {
    typedef double2 T;
};

// Keys weights for offsets -1, 0, 1, 2 at fraction t in [0, 1) (Horner form).
template <typename R>
__device__ inline void keys_weights(R t, R w[4]) {
    const R t2 = t * t, t3 = t2 * t;
    w[0] = R(-0.5) * t3 + t2 - R(0.5) * t;
    w[1] = R(1.5) * t3 - R(2.5) * t2 + R(1);
    w[2] = R(-1.5) * t3 + R(2) * t2 + R(0.5) * t;
    w[3] = R(0.5) * t3 - R(0.5) * t2;
}

// Interpolate ncomp grid planes (plane c at g + c * comp_stride, each
// [n_za][n_az]) at (za, az); out[c * out_stride] = scale * value.
template <typename R, int MODE>
__device__ inline void interp_point(const typename CplxOf<R>::T *__restrict__ g, int64_t comp_stride, int ncomp,
                                    int n_za, int n_az, double dza, double daz, double za, double az, R scale,
                                    typename CplxOf<R>::T *out, int64_t out_stride) {
    typedef typename CplxOf<R>::T C;
    // cell and fractions: integer parts in FP64, fractions in the path's precision
    const double u = za / dza, v = az / daz;
    int j0 = (int)floor(u);
    j0 = j0 < 0 ? 0 : (j0 > n_za - 2 ? n_za - 2 : j0);
    const R t = (R)(u - j0);
    const double kf = floor(v);
    const R s = (R)(v - kf);
    int k0 = (int)kf % n_az;
    if (k0 < 0) k0 += n_az;
    if (MODE == BILINEAR) {
        const int k1 = k0 + 1 == n_az ? 0 : k0 + 1;
        const R w00 = (R(1) - t) * (R(1) - s), w01 = (R(1) - t) * s;
        const R w10 = t * (R(1) - s), w11 = t * s;
        for (int c = 0; c < ncomp; c++) {
            const C *gc = g + c * comp_stride;
            const C g00 = gc[(int64_t)j0 * n_az + k0], g01 = gc[(int64_t)j0 * n_az + k1];
            const C g10 = gc[(int64_t)(j0 + 1) * n_az + k0], g11 = gc[(int64_t)(j0 + 1) * n_az + k1];
            C r;
            r.x = scale * (w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x);
            r.y = scale * (w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y);
            out[c * out_stride] = r;
        }
    } else {
        R wj[4], wk[4];
        keys_weights<R>(t, wj);
        keys_weights<R>(s, wk);
        int kc[4];
        for (int d = 0; d < 4; d++) {
            const int k = k0 - 1 + d;
            kc[d] = k < 0 ? k + n_az : (k >= n_az ? k - n_az : k);
        }
        for (int c = 0; c < ncomp; c++) {
            const C *gc = g + c * comp_stride;
            R accx = 0, accy = 0;
            for (int dj = 0; dj < 4; dj++) {
                const int j = j0 - 1 + dj;
                R rx = 0, ry = 0;  // az-convolved row j
                if (j >= 0 && j < n_za) {
                    const C *row = gc + (int64_t)j * n_az;
                    for (int d = 0; d < 4; d++) {
                        const C q = row[kc[d]];
                        rx += wk[d] * q.x;
                        ry += wk[d] * q.y;
                    }
                } else {
                    // Keys end row: 3 r0 - 3 r1 + r2 from the three rows nearest the end
                    const int e0 = j < 0 ? 0 : n_za - 1, step = j < 0 ? 1 : -1;
                    const R cf[3] = {R(3), R(-3), R(1)};
                    for (int q3 = 0; q3 < 3; q3++) {
                        const C *row = gc + (int64_t)(e0 + q3 * step) * n_az;
                        R qx = 0, qy = 0;
                        for (int d = 0; d < 4; d++) {
                            const C q = row[kc[d]];
                            qx += wk[d] * q.x;
                            qy += wk[d] * q.y;
                        }
                        rx += cf[q3] * qx;
                        ry += cf[q3] * qy;
                    }
                }
                accx += wj[dj] * rx;
                accy += wj[dj] * ry;
            }
            C r;
            r.x = scale * accx;
            r.y = scale * accy;
            out[c * out_stride] = r;
        }
    }
}

}  // namespace mv
