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
    R sq = R(1);
    PolSqrt pm{};
    if (a.idx) {
        const int64_t o = (int64_t)f * a.n_src + a.idx[(int64_t)slot * a.ld_src + m];
        if (a.pol)
            pm = pol_sqrt(a.flux[o], a.flux[o + a.stokes_stride], a.flux[o + 2 * a.stokes_stride],
                          a.flux[o + 3 * a.stokes_stride]);
        else
            sq = (R)sqrt(a.flux[o]);
    }
    for (int b = 0; b < a.n_beam; b++) {
        const C *g = (const C *)a.grid + (int64_t)(b * a.n_freq_grid + f) * ncomp * plane;
        C *ob = out + (int64_t)b * ncomp * a.ld_src;
        interp_point<R, MODE>(g, plane, ncomp, a.n_za, a.n_az, a.dza, a.daz, za, az, sq, ob, a.ld_src);
        if (a.pol)  // B = A M, feed by feed (n_ax = 2: components 2 p and 2 p + 1)
            for (int p = 0; p < a.n_feed; p++) {
                const C a0 = ob[(int64_t)(2 * p) * a.ld_src], a1 = ob[(int64_t)(2 * p + 1) * a.ld_src];
                C o0, o1;
                apply_pol_sqrt<R>(pm, a0.x, a0.y, a1.x, a1.y, o0.x, o0.y, o1.x, o1.y);
                ob[(int64_t)(2 * p) * a.ld_src] = o0;
                ob[(int64_t)(2 * p + 1) * a.ld_src] = o1;
            }
    }
}

// [b][F][P] -> [b][P][Fs] with F = n_freq * ncomp, P = n_za * n_az and the run
// stride Fs = F rounded up to even (16-byte aligned runs), 64 x 64 tiles through LDS.
template <typename C>
__global__ void __launch_bounds__(256) k_grid_interleave(const C *__restrict__ in, int F, int64_t P, C *__restrict__ out) {
    const int Fs = (F + 1) & ~1;
    __shared__ C tile[64][65];
    const int b = blockIdx.z;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const C *src = in + (int64_t)b * F * P;
    C *dst = out + (int64_t)b * Fs * P;
    for (int r = ty; r < 64; r += 4) {
        const int f = f0 + r;
        const int64_t p = p0 + tx;
        if (f < F && p < P) tile[r][tx] = src[(int64_t)f * P + p];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t p = p0 + r;
        const int f = f0 + tx;
        if (f < F && p < P) dst[p * Fs + f] = tile[tx][r];
    }
}

// Row weights of the 4-row za stencil folded onto the grid rows base..base+3:
// Keys' end rows (3 g0 - 3 g1 + g2 beyond either end) become weights on real rows.
template <typename R>
__device__ inline int za_rows_bicubic(int j0, int n_za, R t, R eff[4]) {
    R wj[4];
    keys_weights<R>(t, wj);
    const int base = j0 - 1 < 0 ? 0 : (j0 - 1 > n_za - 4 ? n_za - 4 : j0 - 1);
    for (int q = 0; q < 4; q++) eff[q] = R(0);
    for (int dj = 0; dj < 4; dj++) {
        const int j = j0 - 1 + dj;
        if (j >= 0 && j < n_za) {
            eff[j - base] += wj[dj];
        } else {
            const int e0 = j < 0 ? 0 : n_za - 1, step = j < 0 ? 1 : -1;
            eff[e0 - base] += R(3) * wj[dj];
            eff[e0 + step - base] -= R(3) * wj[dj];
            eff[e0 + 2 * step - base] += wj[dj];
        }
    }
    return base;
}

// Stencil of a source on the grid: the first of its NT rows and columns (rows
// folded at the za ends for bicubic, columns wrapped in az) and the row and
// column weights.
template <typename R, int MODE>
__device__ inline void stencil(double za, double az, const InterpArgs &a, int &rbase, int &kstart, R (&wr)[4],
                               R (&wc)[4]) {
    const double u = za / a.dza, v = az / a.daz;
    int j0 = (int)floor(u);
    j0 = j0 < 0 ? 0 : (j0 > a.n_za - 2 ? a.n_za - 2 : j0);
    const R t = (R)(u - j0);
    const double kf = floor(v);
    const R sfr = (R)(v - kf);
    int k0 = (int)kf % a.n_az;
    if (k0 < 0) k0 += a.n_az;
    if (MODE == BILINEAR) {
        rbase = j0;
        wr[0] = R(1) - t;
        wr[1] = t;
        wc[0] = R(1) - sfr;
        wc[1] = sfr;
        wr[2] = wr[3] = wc[2] = wc[3] = R(0);
        kstart = k0;
    } else {
        rbase = za_rows_bicubic<R>(j0, a.n_za, t, wr);
        keys_weights<R>(sfr, wc);
        kstart = k0 == 0 ? a.n_az - 1 : k0 - 1;
    }
}

// One thread per (slot, visible source): the stencil into the scratch of
// interp_stencil_bytes, packed (rbase << 16 | first column) then the weights
// wr[0..3], wc[0..3] as planes of ld_src.
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_stencil(InterpArgs a, Batch bt) {
    const int slot = blockIdx.y;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = a.count ? a.count[slot] : a.fixed_count;
    if (m >= M) return;
    const int64_t ns = (int64_t)bt.ntb * a.ld_src;
    int rbase, kstart;
    R wr[4], wc[4];
    stencil<R, MODE>(a.za_az[(int64_t)slot * 2 * a.ld_src + m], a.za_az[(int64_t)slot * 2 * a.ld_src + a.ld_src + m],
                     a, rbase, kstart, wr, wc);
    int32_t *rc = (int32_t *)a.stencil;
    R *w = (R *)(rc + ns);
    rc[(int64_t)slot * a.ld_src + m] = (rbase << 16) | kstart;
    for (int j = 0; j < 4; j++) {
        w[((int64_t)slot * 8 + j) * a.ld_src + m] = wr[j];
        w[((int64_t)slot * 8 + 4 + j) * a.ld_src + m] = wc[j];
    }
}

// A group of LPS lanes per (visible source, time slot of the batch, 4 channels
// of the batch): a tap's interleaved run T[b][j][k][f .. f + 3][0 .. ncomp) is
// 4 ncomp complex values, and lane l of the group reads its l-th 16-byte piece
// (two complex64 or one complex128), so a wave's load covers whole runs of
// 64 / LPS sources.  The group reads the source's stencil from the scratch
// k_stencil wrote (ST), or every lane forms it.
template <typename R, int MODE, int NCOMP, bool ST>
__global__ void __launch_bounds__(256) k_interp_tf(InterpArgs a, Batch bt) {
    typedef typename CplxOf<R>::T C;
    constexpr int FG = 4;                            // channels per group
    constexpr int PER = 16 / sizeof(C);              // complex values per lane (16 bytes)
    constexpr int LPS = FG * NCOMP / PER;            // lanes per source
    // XCD-aware block order: workgroups go to the 8 XCDs round-robin by linear id,
    // so each XCD is given one contiguous range of (channel group, slot, source
    // block) work; neighbouring (sky-cell ordered) sources then share one L2 and
    // the grid lines they have in common are fetched into it once.
    const uint32_t gx = gridDim.x, gy = gridDim.y;
    const uint32_t total = gx * gy * gridDim.z;
    const uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t xq = total / 8, xr = total % 8, xcd = lin % 8;
    const uint32_t task = xcd * xq + (xcd < xr ? xcd : xr) + lin / 8;
    const uint32_t bx = task % gx;
    const int slot = (int)((task / gx) % gy);
    const int fg = (int)(task / (gx * gy)) * FG;    // first channel of the group, relative to the batch
    const int l = threadIdx.x % LPS;
    const int64_t m = (int64_t)bx * (blockDim.x / LPS) + threadIdx.x / LPS;
    const int64_t M = a.count ? a.count[slot] : a.fixed_count;
    if (m >= M || fg >= bt.nfb) return;
    const int nf = bt.nfb - fg < FG ? bt.nfb - fg : FG;
    constexpr int NT = MODE == BILINEAR ? 2 : 4;
    R wr[4], wc[4];
    int rbase, kstart;
    if constexpr (ST) {
        const int32_t *rc = (const int32_t *)a.stencil;
        const R *w = (const R *)(rc + (int64_t)bt.ntb * a.ld_src);
        const int32_t p = rc[(int64_t)slot * a.ld_src + m];
        rbase = (int)((uint32_t)p >> 16);
        kstart = p & 0xffff;
#pragma unroll
        for (int j = 0; j < NT; j++) {
            wr[j] = w[((int64_t)slot * 8 + j) * a.ld_src + m];
            wc[j] = w[((int64_t)slot * 8 + 4 + j) * a.ld_src + m];
        }
    } else {
        stencil<R, MODE>(a.za_az[(int64_t)slot * 2 * a.ld_src + m], a.za_az[(int64_t)slot * 2 * a.ld_src + a.ld_src + m],
                         a, rbase, kstart, wr, wc);
    }
    int kc[NT];
#pragma unroll
    for (int d = 0; d < NT; d++) kc[d] = kstart + d >= a.n_az ? kstart + d - a.n_az : kstart + d;
    const int F = (a.n_freq_grid * NCOMP + 1) & ~1;  // run stride of one grid point (all channels, even)
    const int fabs0 = bt.f0 + fg;
    // this lane's elements e = l PER + p of the group's run: channel q = e / NCOMP, component e % NCOMP
    const int e0 = l * PER;
    const bool live = e0 / NCOMP < nf;
    R sq[PER];
    for (int p = 0; p < PER; p++) {
        const int q = (e0 + p) / NCOMP;
        sq[p] = R(1);
        if (a.idx && q < nf && !a.pol)
            sq[p] = (R)sqrt(a.flux[(int64_t)(fabs0 + q) * a.n_src + a.idx[(int64_t)slot * a.ld_src + m]]);
    }
    // polarised sky: the square root of this lane's channel's brightness matrix
    // (NCOMP is even then, so a lane's elements belong to one channel)
    PolSqrt pm{};
    if (a.pol && e0 / NCOMP < nf) {
        const int64_t o = (int64_t)(fabs0 + e0 / NCOMP) * a.n_src + a.idx[(int64_t)slot * a.ld_src + m];
        pm = pol_sqrt(a.flux[o], a.flux[o + a.stokes_stride], a.flux[o + 2 * a.stokes_stride],
                      a.flux[o + 3 * a.stokes_stride]);
    }
    for (int b = 0; b < a.n_beam; b++) {
        const C *T = (const C *)a.grid + (int64_t)b * a.n_za * a.n_az * F + (int64_t)fabs0 * NCOMP + e0;
        R ax[PER], ay[PER];
        for (int p = 0; p < PER; p++) ax[p] = ay[p] = R(0);
        if (live) {
#pragma unroll
            for (int dr = 0; dr < NT; dr++) {
                const int64_t row = (int64_t)(rbase + dr) * a.n_az;
#pragma unroll
                for (int d = 0; d < NT; d++) {
                    const R w = wr[dr] * wc[d];
                    const C *tp = T + (row + kc[d]) * F;
                    C g[PER];
                    if constexpr (PER == 2) {
                        const float4 q4 = *(const float4 *)tp;
                        g[0] = make_float2(q4.x, q4.y);
                        g[PER - 1] = make_float2(q4.z, q4.w);
                    } else {
                        g[0] = *tp;
                    }
#pragma unroll
                    for (int p = 0; p < PER; p++) {
                        ax[p] += w * g[p].x;
                        ay[p] += w * g[p].y;
                    }
                }
            }
        }
        if (a.pol) {
            // B = A M per feed: components 2 p + k, k = 0, 1 of one channel
            if constexpr (PER == 2) {
                R o0x, o0y, o1x, o1y;
                apply_pol_sqrt<R>(pm, ax[0], ay[0], ax[1], ay[1], o0x, o0y, o1x, o1y);
                ax[0] = o0x;
                ay[0] = o0y;
                ax[1] = o1x;
                ay[1] = o1y;
            } else {
                // one component per lane: the other axis of the feed is in the neighbouring lane
                const R px = __shfl_xor(ax[0], 1), py = __shfl_xor(ay[0], 1);
                R o0x, o0y, o1x, o1y;
                if ((e0 & 1) == 0) {
                    apply_pol_sqrt<R>(pm, ax[0], ay[0], px, py, o0x, o0y, o1x, o1y);
                    ax[0] = o0x;
                    ay[0] = o0y;
                } else {
                    apply_pol_sqrt<R>(pm, px, py, ax[0], ay[0], o0x, o0y, o1x, o1y);
                    ax[0] = o1x;
                    ay[0] = o1y;
                }
            }
            for (int p = 0; p < PER; p++) sq[p] = R(1);
        }
        for (int p = 0; p < PER; p++) {
            const int e = e0 + p, q = e / NCOMP, c = e % NCOMP;
            if (q >= nf) continue;
            const int inst = slot * bt.nfb + fg + q;
            C r;
            r.x = sq[p] * ax[p];
            r.y = sq[p] * ay[p];
            ((C *)a.A)[(((int64_t)inst * a.n_beam + b) * NCOMP + c) * a.ld_src + m] = r;
        }
    }
}

template <typename R, int MODE>
hipError_t launch_tf_mode(const InterpArgs &a, const Batch &bt, hipStream_t s) {
    const int ncomp = a.n_feed * a.n_ax;
    const int lps = 4 * ncomp * (int)sizeof(typename CplxOf<R>::T) / 16;  // lanes per source
    const int sources_per_block = 256 / lps;
    dim3 g((unsigned)((a.max_m + sources_per_block - 1) / sources_per_block), bt.n_inst / bt.nfb,
           (unsigned)((bt.nfb + 3) / 4));
    if (a.stencil) {
        k_stencil<R, MODE><<<dim3((unsigned)((a.max_m + 255) / 256), (unsigned)bt.ntb), 256, 0, s>>>(a, bt);
        if (ncomp == 4)
            k_interp_tf<R, MODE, 4, true><<<g, 256, 0, s>>>(a, bt);
        else if (ncomp == 2)
            k_interp_tf<R, MODE, 2, true><<<g, 256, 0, s>>>(a, bt);
        else
            k_interp_tf<R, MODE, 1, true><<<g, 256, 0, s>>>(a, bt);
    } else {
        if (ncomp == 4)
            k_interp_tf<R, MODE, 4, false><<<g, 256, 0, s>>>(a, bt);
        else if (ncomp == 2)
            k_interp_tf<R, MODE, 2, false><<<g, 256, 0, s>>>(a, bt);
        else
            k_interp_tf<R, MODE, 1, false><<<g, 256, 0, s>>>(a, bt);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_interleave(int prec, const void *grid, int n_beam, int n_freq, int ncomp, int n_za, int n_az,
                                  void *T, hipStream_t s) {
    const int F = n_freq * ncomp;
    const int64_t P = (int64_t)n_za * n_az;
    dim3 g((unsigned)((P + 63) / 64), (unsigned)((F + 63) / 64), (unsigned)n_beam);
    if (prec == P64)
        k_grid_interleave<double2><<<g, 256, 0, s>>>((const double2 *)grid, F, P, (double2 *)T);
    else
        k_grid_interleave<float2><<<g, 256, 0, s>>>((const float2 *)grid, F, P, (float2 *)T);
    return hipGetLastError();
}

hipError_t launch_interp_tf(int prec, int mode, const InterpArgs &a, const Batch &bt, hipStream_t s) {
    if (bt.n_inst <= 0 || a.max_m <= 0) return hipSuccess;
    if (a.n_za < 4 || a.n_za >= 65536 || a.n_az >= 65536) return hipErrorInvalidValue;
    if (prec == P64)
        return mode == BILINEAR ? launch_tf_mode<double, BILINEAR>(a, bt, s) : launch_tf_mode<double, BICUBIC>(a, bt, s);
    return mode == BILINEAR ? launch_tf_mode<float, BILINEAR>(a, bt, s) : launch_tf_mode<float, BICUBIC>(a, bt, s);
}

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
