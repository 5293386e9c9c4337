// Sky geometry on the device: Eq. (xeq), Eq. (rotation), the topocentric
// rotation of Alg. 2 step (i) and the order-preserving horizon compaction.
//
// Compaction is three passes per (time batch, source chunk):
//   count   : one wave64 ballot per 64 sources, popcount, per-block sums;
//   scan    : exclusive prefix over the block sums of every time;
//   scatter : recompute the rotation (cheaper than storing it), place each
//             visible source at block offset + wave offset + mbcnt lane rank.
// The result lists visible sources in ascending index order, so it is
// deterministic and equal to a sequential filter.
//
// Before that, the catalogue is put into a spatially coherent order once per
// call (a stable counting sort by sky cell: the face of the enclosing cube and
// a 16 x 16 Morton cell on it), so that consecutive visible sources -- and the
// threads that interpolate the beam for them -- fall on nearby grid points.
// The sky arrays then follow that order; the index lists hold the original
// source numbers, so fluxes are read unchanged.
#include "internal.h"

namespace mv {

namespace {

constexpr int kSkyBlock = 256;

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of `mask` below this lane.
__device__ inline int rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

constexpr int kCells = 6 * 256;  // cube faces x 16 x 16 Morton cells

__device__ inline int spread4(int v) {  // 4 bits -> even bit positions
    v = (v | (v << 2)) & 0x33;
    v = (v | (v << 1)) & 0x55;
    return v;
}

__device__ inline int sky_cell(double x, double y, double z) {
    const double ax = fabs(x), ay = fabs(y), az = fabs(z);
    int face;
    double u, v, m;
    if (ax >= ay && ax >= az) {
        face = x >= 0 ? 0 : 1, u = y, v = z, m = ax;
    } else if (ay >= az) {
        face = y >= 0 ? 2 : 3, u = x, v = z, m = ay;
    } else {
        face = z >= 0 ? 4 : 5, u = x, v = y, m = az;
    }
    int iu = (int)((u / m + 1.0) * 8.0), iv = (int)((v / m + 1.0) * 8.0);
    iu = iu < 0 ? 0 : (iu > 15 ? 15 : iu);
    iv = iv < 0 ? 0 : (iv > 15 ? 15 : iv);
    return face * 256 + (spread4(iu) | (spread4(iv) << 1));
}

// Eq. (xeq) in input order, each source's sky cell, and per-block cell counts.
__global__ void __launch_bounds__(kSkyBlock) k_xeq_cells(const double *__restrict__ radec, int64_t n,
                                                         double *__restrict__ xeq_in, int64_t ld,
                                                         int16_t *__restrict__ cell, int32_t *__restrict__ hist) {
    __shared__ int h[kCells];
    for (int c = threadIdx.x; c < kCells; c += kSkyBlock) h[c] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kSkyBlock + threadIdx.x;
    if (i < n) {
        double sr, cr, sd, cd;
        sincos(radec[i], &sr, &cr);
        sincos(radec[n + i], &sd, &cd);
        const double x = cr * cd, y = sr * cd, z = sd;
        xeq_in[i] = x;
        xeq_in[ld + i] = y;
        xeq_in[2 * ld + i] = z;
        const int c = sky_cell(x, y, z);
        cell[i] = (int16_t)c;
        atomicAdd(&h[c], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kCells; c += kSkyBlock) hist[(int64_t)blockIdx.x * kCells + c] = h[c];
}

// hist[b][c] -> first position of block b's cell-c sources in the cell-major
// order, in three passes over chunks of `chunk` blocks (a multiple of 8 giving
// at most 256 chunks) so that every pass reads whole rows of hist (coalesced)
// and all CUs take part:
//   k_cell_chunk_sums:    part[ch][c] = cell-c count over the blocks of chunk ch;
//   k_cell_chunk_offsets: cell totals scanned (exclusive), then each cell's
//                         chunks scanned on top: part[ch][c] = first position of
//                         chunk ch's cell-c sources (one workgroup);
//   k_cell_apply:         each chunk walks its blocks, hist[b][c] = position.
__host__ __device__ inline int cell_chunk(int nblk) { return ((nblk + 255) / 256 + 7) / 8 * 8; }

__global__ void __launch_bounds__(256) k_cell_chunk_sums(const int32_t *__restrict__ hist, int nblk, int chunk,
                                                         int32_t *__restrict__ part) {
    const int ch = blockIdx.x;
    const int b0 = ch * chunk, b1 = nblk < b0 + chunk ? nblk : b0 + chunk;
    for (int c = threadIdx.x; c < kCells; c += 256) {
        int run = 0;
#pragma unroll 8
        for (int b = b0; b < b1; b++) run += hist[(int64_t)b * kCells + c];
        part[(int64_t)ch * kCells + c] = run;
    }
}

__global__ void __launch_bounds__(1024) k_cell_chunk_offsets(int32_t *__restrict__ part, int nchunk) {
    __shared__ int tot[kCells];
    __shared__ int wsum[1024 / kWave];
    for (int c = threadIdx.x; c < kCells; c += 1024) {
        int run = 0;
#pragma unroll 16
        for (int ch = 0; ch < nchunk; ch++) run += part[(int64_t)ch * kCells + c];
        tot[c] = run;
    }
    __syncthreads();
    // exclusive scan of the cell totals (kCells <= 2 x 1024)
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int carry = 0;
    for (int base = 0; base < kCells; base += 1024) {
        const int c = base + threadIdx.x;
        const int v = c < kCells ? tot[c] : 0;
        int x = v;
        for (int d = 1; d < kWave; d <<= 1) {
            const int y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        int woff = 0;
        for (int q = 0; q < w; q++) woff += wsum[q];
        const int excl = carry + woff + x - v;
        int block_total = 0;
        for (int q = 0; q < 1024 / kWave; q++) block_total += wsum[q];
        __syncthreads();
        if (c < kCells) tot[c] = excl;
        carry += block_total;
        __syncthreads();
    }
    for (int c = threadIdx.x; c < kCells; c += 1024) {
        int run = tot[c];
        for (int ch = 0; ch < nchunk; ch++) {
            const int v = part[(int64_t)ch * kCells + c];
            part[(int64_t)ch * kCells + c] = run;
            run += v;
        }
    }
}

__global__ void __launch_bounds__(256) k_cell_apply(int32_t *__restrict__ hist, int nblk, int chunk,
                                                    const int32_t *__restrict__ part) {
    const int ch = blockIdx.x;
    const int b0 = ch * chunk, b1 = nblk < b0 + chunk ? nblk : b0 + chunk;
    for (int c = threadIdx.x; c < kCells; c += 256) {
        int run = part[(int64_t)ch * kCells + c];
#pragma unroll 8
        for (int b = b0; b < b1; b++) {
            const int v = hist[(int64_t)b * kCells + c];
            hist[(int64_t)b * kCells + c] = run;
            run += v;
        }
    }
}

// Stable scatter into cell order: rank among earlier sources of the same cell in the block.
__global__ void __launch_bounds__(kSkyBlock) k_cell_scatter(const double *__restrict__ xeq_in, int64_t n, int64_t ld,
                                                            const int16_t *__restrict__ cell,
                                                            const int32_t *__restrict__ hist, double *__restrict__ xeq,
                                                            int32_t *__restrict__ perm) {
    __shared__ int16_t kc[kSkyBlock];
    const int64_t i = (int64_t)blockIdx.x * kSkyBlock + threadIdx.x;
    const int c = i < n ? cell[i] : -1;
    kc[threadIdx.x] = (int16_t)c;
    __syncthreads();
    if (i >= n) return;
    int rank = 0;
    for (int j = 0; j < (int)threadIdx.x; j++) rank += kc[j] == c;
    const int64_t pos = hist[(int64_t)blockIdx.x * kCells + c] + rank;
    xeq[pos] = xeq_in[i];
    xeq[ld + pos] = xeq_in[ld + i];
    xeq[2 * ld + pos] = xeq_in[2 * ld + i];
    perm[pos] = (int32_t)i;
}

__global__ void k_xeq(const double *__restrict__ radec, int64_t n, double *__restrict__ xeq, int64_t ld) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sr, cr, sd, cd;
    sincos(radec[i], &sr, &cr);
    sincos(radec[n + i], &sd, &cd);
    xeq[i] = cr * cd;
    xeq[ld + i] = sr * cd;
    xeq[2 * ld + i] = sd;
}

// R(t) of Eq. (rotation) with hour angle H = -LST and latitude l.
__global__ void k_rotmats(const double *__restrict__ lsts, int n_time, double lat, double *__restrict__ rot) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_time) return;
    double sH, cH, sl, cl;
    sincos(-lsts[t], &sH, &cH);
    sincos(lat, &sl, &cl);
    double *r = rot + 9 * t;
    r[0] = sH;
    r[1] = cH;
    r[2] = 0.0;
    r[3] = -sl * cH;
    r[4] = sl * sH;
    r[5] = cl;
    r[6] = cl * cH;
    r[7] = -cl * sH;
    r[8] = sl;
}

// One block: centre the antennas on their mean (a common offset cancels in
// every baseline), sanitise beam indices, and flag invalid inputs.  The flux
// check runs grid-wide in k_check_flux.
__global__ void k_prep_ant(const double *__restrict__ antpos, int n_ant, const int32_t *__restrict__ beam_idx,
                           int n_beam, double *__restrict__ antc, int32_t *__restrict__ bidx, int32_t *flags) {
    __shared__ double red[3][kSkyBlock];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    int bad = 0;
    for (int a = threadIdx.x; a < n_ant; a += blockDim.x) {
        double x = antpos[3 * a], y = antpos[3 * a + 1], z = antpos[3 * a + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) bad |= FLAG_BAD_ANTPOS;
        s0 += x;
        s1 += y;
        s2 += z;
        int b = beam_idx ? beam_idx[a] : 0;
        if (b < 0 || b >= n_beam) {
            bad |= FLAG_BAD_BEAM_IDX;
            b = b < 0 ? 0 : n_beam - 1;
        }
        bidx[a] = b;
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = kSkyBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; c++) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    double inv = n_ant > 0 ? 1.0 / n_ant : 0.0;
    double m0 = red[0][0] * inv, m1 = red[1][0] * inv, m2 = red[2][0] * inv;
    for (int a = threadIdx.x; a < n_ant; a += blockDim.x) {
        antc[3 * a] = antpos[3 * a] - m0;
        antc[3 * a + 1] = antpos[3 * a + 1] - m1;
        antc[3 * a + 2] = antpos[3 * a + 2] - m2;
    }
    if (bad) atomicOr(flags, bad);
}

__global__ void k_check_flux(const double *__restrict__ flux, int64_t n, int pol, int32_t *flags) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double f = flux[i];
        if (!(f >= 0.0) || !isfinite(f)) bad = true;
        if (pol) {
            // a physical brightness matrix: Q^2 + U^2 + V^2 <= I^2 (relative 1e-9)
            const double q = flux[n + i], u = flux[2 * n + i], v = flux[3 * n + i];
            if (!isfinite(q) || !isfinite(u) || !isfinite(v) || !(q * q + u * u + v * v <= f * f * (1.0 + 1e-9)))
                bad = true;
        }
    }
    unsigned long long m = __ballot(bad);
    if (m && lane_id() == __ffsll((long long)m) - 1) atomicOr(flags, FLAG_BAD_FLUX);
}

// Up-component of R(t) X_eq for source n.
__device__ inline double up_of(const double *r, const double *__restrict__ xeq, int64_t ld, int64_t n) {
    return r[6] * xeq[n] + r[7] * xeq[ld + n] + r[8] * xeq[2 * ld + n];
}

__global__ void __launch_bounds__(kSkyBlock) k_sky_count(SkyBufs b, int t0, int64_t c0, int64_t nsrc, int nblk) {
    __shared__ int wsum[kSkyBlock / kWave];
    const int ts = blockIdx.y;
    const double *r = b.rot + 9 * (t0 + ts);
    int64_t j = (int64_t)blockIdx.x * kSkyBlock + threadIdx.x;
    bool vis = false;
    if (j < nsrc) vis = up_of(r, b.xeq, b.ld_xeq, c0 + j) > 0.0;
    unsigned long long m = __ballot(vis);
    int w = threadIdx.x / kWave;
    if (lane_id() == 0) wsum[w] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < kSkyBlock / kWave; i++) s += wsum[i];
        b.blk_count[(int64_t)ts * nblk + blockIdx.x] = s;
    }
}

// Exclusive scan of the block counts of one time slot; one 1024-thread block per slot.
__global__ void __launch_bounds__(1024) k_sky_scan(SkyBufs b, int nblk) {
    __shared__ int wtot[1024 / kWave];
    __shared__ int carry_s;
    const int ts = blockIdx.x;
    const int32_t *in = b.blk_count + (int64_t)ts * nblk;
    int32_t *out = b.blk_off + (int64_t)ts * nblk;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    for (int base = 0; base < nblk; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < nblk ? in[i] : 0;
        int x = v;  // inclusive scan inside the wave
        for (int d = 1; d < kWave; d <<= 1) {
            int y = __shfl_up(x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) wtot[w] = x;
        __syncthreads();
        if (w == 0) {
            int t = lane < 1024 / kWave ? wtot[lane] : 0;
            for (int d = 1; d < kWave; d <<= 1) {
                int y = __shfl_up(t, d, kWave);
                if (lane >= d) t += y;
            }
            if (lane < 1024 / kWave) wtot[lane] = t;  // inclusive prefix of wave totals
        }
        __syncthreads();
        int carry = carry_s;
        int wave_excl = w > 0 ? wtot[w - 1] : 0;
        if (i < nblk) out[i] = carry + wave_excl + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + wtot[1024 / kWave - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.count[ts] = carry_s;
}

__global__ void __launch_bounds__(kSkyBlock) k_sky_scatter(SkyBufs b, int t0, int64_t c0, int64_t nsrc, int nblk) {
    __shared__ int wsum[kSkyBlock / kWave];
    const int ts = blockIdx.y;
    const double *r = b.rot + 9 * (t0 + ts);
    const int64_t ld = b.ld_src;
    int64_t j = (int64_t)blockIdx.x * kSkyBlock + threadIdx.x;
    double e = 0.0, nn = 0.0, u = 0.0;
    bool vis = false;
    if (j < nsrc) {
        int64_t n = c0 + j;
        double x = b.xeq[n], y = b.xeq[b.ld_xeq + n], z = b.xeq[2 * b.ld_xeq + n];
        e = r[0] * x + r[1] * y + r[2] * z;
        nn = r[3] * x + r[4] * y + r[5] * z;
        u = r[6] * x + r[7] * y + r[8] * z;
        vis = u > 0.0;
    }
    unsigned long long m = __ballot(vis);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int woff = 0;
    for (int i = 0; i < w; i++) woff += wsum[i];
    if (vis) {
        int64_t o = b.blk_off[(int64_t)ts * nblk + blockIdx.x] + woff + rank_below(m);
        b.idx[ts * ld + o] = b.perm ? b.perm[c0 + j] : (int32_t)(c0 + j);
        double *sh = b.s_hat + (int64_t)ts * 3 * ld;
        sh[o] = e;
        sh[ld + o] = nn;
        sh[2 * ld + o] = u;
        double za = atan2(hypot(e, nn), u);
        double az = atan2(e, nn);
        if (az < 0.0) az += 2.0 * M_PI;
        if (az >= 2.0 * M_PI) az -= 2.0 * M_PI;
        double *zz = b.za_az + (int64_t)ts * 2 * ld;
        zz[o] = za;
        zz[ld + o] = az;
    }
}

}  // namespace

hipError_t launch_xeq(const double *radec, int64_t n_src, double *xeq, int64_t ld, hipStream_t s) {
    if (n_src <= 0) return hipSuccess;
    k_xeq<<<(unsigned)((n_src + 255) / 256), 256, 0, s>>>(radec, n_src, xeq, ld);
    return hipGetLastError();
}

hipError_t launch_xeq_sorted(const double *radec, int64_t n_src, int64_t ld, SortBufs sb, double *xeq, hipStream_t s) {
    if (n_src <= 0) return hipSuccess;
    const int nblk = (int)((n_src + kSkyBlock - 1) / kSkyBlock);
    k_xeq_cells<<<nblk, kSkyBlock, 0, s>>>(radec, n_src, sb.xeq_in, ld, sb.cell, sb.hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // chunk partials after the per-block counts (sort_hist_entries leaves room)
    const int chunk = cell_chunk(nblk);
    const int nchunk = (nblk + chunk - 1) / chunk;
    int32_t *part = sb.hist + (int64_t)nblk * kCells;
    k_cell_chunk_sums<<<nchunk, 256, 0, s>>>(sb.hist, nblk, chunk, part);
    k_cell_chunk_offsets<<<1, 1024, 0, s>>>(part, nchunk);
    k_cell_apply<<<nchunk, 256, 0, s>>>(sb.hist, nblk, chunk, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_cell_scatter<<<nblk, kSkyBlock, 0, s>>>(sb.xeq_in, n_src, ld, sb.cell, sb.hist, xeq, sb.perm);
    return hipGetLastError();
}

int64_t sort_hist_entries(int64_t max_src) {
    const int64_t nblk = (max_src + kSkyBlock - 1) / kSkyBlock;
    return (nblk + (nblk + 7) / 8) * kCells;  // per-block counts, then per-chunk partials (chunks of >= 8 blocks)
}

hipError_t launch_rotmats(const double *lsts, int32_t n_time, double latitude, double *rot, hipStream_t s) {
    if (n_time <= 0) return hipSuccess;
    k_rotmats<<<(n_time + 63) / 64, 64, 0, s>>>(lsts, n_time, latitude, rot);
    return hipGetLastError();
}

hipError_t launch_prep_inputs(const double *antpos, int32_t n_ant, const int32_t *beam_idx, int32_t n_beam,
                              const double *flux, int64_t n_flux, int pol, double *antc, int32_t *bidx,
                              int32_t *flags, hipStream_t s) {
    k_prep_ant<<<1, kSkyBlock, 0, s>>>(antpos, n_ant, beam_idx, n_beam, antc, bidx, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_flux <= 0 || !flux) return e;
    int64_t blocks = (n_flux + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_check_flux<<<(unsigned)blocks, 256, 0, s>>>(flux, n_flux, pol, flags);
    return hipGetLastError();
}

hipError_t launch_sky(const SkyBufs &b, int32_t t0, int32_t ntb, int64_t c0, int64_t nsrc_chunk, hipStream_t s) {
    if (ntb <= 0) return hipSuccess;
    int nblk = (int)((nsrc_chunk + kSkyBlock - 1) / kSkyBlock);
    if (nblk == 0) nblk = 1;
    dim3 g(nblk, ntb);
    k_sky_count<<<g, kSkyBlock, 0, s>>>(b, t0, c0, nsrc_chunk, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sky_scan<<<ntb, 1024, 0, s>>>(b, nblk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sky_scatter<<<g, kSkyBlock, 0, s>>>(b, t0, c0, nsrc_chunk, nblk);
    return hipGetLastError();
}

}  // namespace mv
