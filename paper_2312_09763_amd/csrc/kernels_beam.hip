// Alg. 2 step (ii): beam (Jones terms) at the visible sources' (za, az) on an
// az/za grid whose pole is the zenith (Sec. 3.4); the interpolants are in
// beam_interp.h.  One thread per (visible source, instance); the taps are read
// through the L2 / MALL (a 0.5 deg polarised channel is 4.2 MB in complex64).
// When the product forms Z itself, the output is B = sqrt(I) A.
#include "beam_interp.h"

namespace mv {

namespace {

template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_interp(InterpArgs a, Batch bt) {
    typedef typename CplxOf<R>::T C;
    const int inst = blockIdx.y;
    const int slot = inst / bt.nfb;
    const int f = bt.f0 + inst % bt.nfb;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = a.count ? a.count[slot] : a.fixed_count;
    if (m >= M) return;
    const double za = a.za_az[(int64_t)slot * 2 * a.ld_src + m];
    const double az = a.za_az[(int64_t)slot * 2 * a.ld_src + a.ld_src + m];
    const int ncomp = a.n_feed * a.n_ax;
    const int64_t plane = (int64_t)a.n_za * a.n_az;
    C *out = (C *)a.A + (int64_t)inst * a.n_beam * ncomp * a.ld_src + m;
    const R sq = a.idx ? (R)sqrt(a.flux[(int64_t)f * a.n_src + a.idx[(int64_t)slot * a.ld_src + m]]) : R(1);
    for (int b = 0; b < a.n_beam; b++) {
        const C *g = (const C *)a.grid + (int64_t)(b * a.n_freq_grid + f) * ncomp * plane;
        interp_point<R, MODE>(g, plane, ncomp, a.n_za, a.n_az, a.dza, a.daz, za, az, sq, out + (int64_t)b * ncomp * a.ld_src,
                              a.ld_src);
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
