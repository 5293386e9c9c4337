// Alg. 2 steps (iii)-(v) in one kernel: Z of Eq. (littlez) is formed in LDS,
// tile by tile, and consumed there by the MFMA product of Eq. (zz); Z never
// reaches HBM.
//
// A 512-thread workgroup holds a (instance, k-split, lower super-tile I >= J)
// work item of the persistent work list (same list as the unfused product).
// Waves 0-3 are consumers: each owns a 64 x 64 wave tile of the 128 x 128
// super-tile and runs the MFMA products exactly like the unfused kernel.
// Waves 4-7 are producers: for the next stage of KC = 32 complex columns
// (KC / n_ax sources) they compute, for every antenna of row blocks I and J,
//   p = (nu/c) x_a . s_m in cycles (FP64),  r = p - rint(p),
//   F = cospi(2r) - i sinpi(2r)           (FP32 sincospi),
//   Z[(a, p)][(m, k)] = B_{beam(a), p, k}(m) F,  B = sqrt(I) A (from the beam step),
// and write it to the other LDS buffer (complex64 on FP32; bf16 hi / lo planes
// on BF16X3).  One barrier per stage swaps the buffers, so the VALU work of
// the producers overlaps the matrix-core work of the consumers on every SIMD
// (one wave of each kind per SIMD).
//
// Per item, the scaled antenna positions (nu/c) x_a and beam indices of the
// item's rows are staged once in LDS; per stage, each producer thread's
// source direction and beam values were loaded into registers during the
// previous stage, so no producer waits on device memory in its inner loop.
// Per source the item reads 24 B of direction and 8 n_feed n_ax B of beam;
// everything else is arithmetic.  Partials go to the same slots as the
// unfused product and are summed by k_reduce.
#include "internal.h"

namespace mv {

namespace {

constexpr int kST = 128, kWT = 64, kKC = 32, kTI = 4;

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }

// packed (hi, lo) bf16 words of one complex64 value
__device__ inline void split2(float re, float im, uint32_t &hi, uint32_t &lo) {
    const uint32_t hr = bf16_rne(re), hm = bf16_rne(im);
    hi = hr | (hm << 16);
    lo = bf16_rne(re - bf16_to_f(hr)) | (bf16_rne(im - bf16_to_f(hm)) << 16);
}

__device__ inline u32x4 bf16_rot(u32x4 v) {
    u32x4 r;
    for (int q = 0; q < 4; q++) r[q] = __builtin_amdgcn_alignbit(v[q], v[q], 16) ^ 0x80000000u;
    return r;
}

template <int PREC>
struct FL {
    static constexpr int EBP = PREC == PB3 ? 4 : 8;      // bytes per complex per plane
    static constexpr int PLANES = PREC == PB3 ? 2 : 1;
    static constexpr int PLANEB = kKC * EBP;              // bytes of one plane of a staged row
    static constexpr int RS = kKC * EBP * PLANES + 16;    // LDS row stride
    static constexpr int BUF = 2 * kST * RS;              // one stage buffer (rows of I and J)
    static constexpr int TAB = 2 * kST;                   // antenna table entries (rows of I and J, n_feed = 1)
};

struct AntEntry {
    double ux, uy, uz;  // (nu / c) x_a
    int b;              // beam index, -1 for padding rows
    int pad;
};

template <int PREC, int NF, int NX>
__global__ void __launch_bounds__(512, 1) k_herk_fused(FusedArgs a) {
    typedef FL<PREC> L;
    constexpr int RS = L::RS;
    constexpr int NC = NF * NX;       // beam components per source
    constexpr int SPS = kKC / NX;     // sources per stage
    constexpr int APB = kST / NF;     // antennas per row block
    constexpr int NG = 256 / SPS;     // producer thread groups (one source per thread)
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * L::BUF];
    __shared__ AntEntry tab[2 * APB];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const bool consumer = wave < 4;
    const int wr = (wave & 3) >> 1, wc = wave & 1;
    const int l16 = lane & 15, lk = lane >> 4;
    const int Np = a.n_rows_pad;
    const int nb = Np / kST;
    const int n_st = nb * (nb + 1) / 2;
    const int total = a.work[a.n_inst];
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    // producer thread roles
    const int pt = tid - 256;
    const int msl = pt % SPS, g = pt / SPS;

    for (int item = slot_x; item < total; item += a.grid) {
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work[mid] <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int inst = lo;
        const int local = item - a.work[inst];
        const int s = local / n_st;
        int st = local % n_st;
        int I = 0;
        while (st > I) {
            st -= I + 1;
            I++;
        }
        const int J = st;
        const bool diag = I == J;
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.ksplit / NX;
        const int64_t m_begin = (int64_t)s * ms_per_split;
        const int64_t m_end = m_begin + ms_per_split < M ? m_begin + ms_per_split : M;
        const int n_stage = (int)((m_end - m_begin + SPS - 1) / SPS);
        const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
        const float2 *Bm = (const float2 *)a.B + (int64_t)inst * a.n_beam * NC * a.ld_src;
        const int na_tot = (diag ? 1 : 2) * APB;

        // antenna table of this item's rows
        {
            const double nu_c = a.freqs[f] / kSpeedOfLight;
            for (int as = tid; as < na_tot; as += 512) {
                const int ant = as < APB ? I * APB + as : J * APB + (as - APB);
                AntEntry e;
                if (ant < a.n_ant) {
                    e.ux = nu_c * a.antc[3 * ant];
                    e.uy = nu_c * a.antc[3 * ant + 1];
                    e.uz = nu_c * a.antc[3 * ant + 2];
                    e.b = a.bidx[ant];
                } else {
                    e.ux = e.uy = e.uz = 0.0;
                    e.b = -1;
                }
                e.pad = 0;
                tab[as] = e;
            }
        }

        // producer registers: direction and beam of this thread's source in the next stage
        double sx = 0.0, sy = 0.0, sz = 0.0;
        float2 w[NC];
        bool live = false;
        int64_t m_cur = 0;
        auto fetch = [&](int stage) {
            m_cur = m_begin + (int64_t)stage * SPS + msl;
            live = stage < n_stage && m_cur < m_end;
            if (live) {
                sx = sh[m_cur];
                sy = sh[a.ld_src + m_cur];
                sz = sh[2 * a.ld_src + m_cur];
                if (a.n_beam == 1)
                    for (int c = 0; c < NC; c++) w[c] = Bm[(int64_t)c * a.ld_src + m_cur];
            }
        };

        // ---- producer: form the Z rows of blocks I (and J) for one stage
        auto produce = [&](unsigned char *buf) {
            const bool lv = live;
            const double x0 = sx, x1 = sy, x2 = sz;
            const int64_t m = m_cur;
            float2 wl[NC];
            for (int c = 0; c < NC; c++) wl[c] = w[c];
            int cur_b = a.n_beam == 1 ? 0 : -1;
            for (int as = g; as < na_tot; as += NG) {
                const AntEntry e = tab[as];
                float2 z[NC];
                for (int c = 0; c < NC; c++) z[c] = make_float2(0.f, 0.f);
                if (lv && e.b >= 0) {
                    if (e.b != cur_b) {
                        for (int c = 0; c < NC; c++) wl[c] = Bm[((int64_t)e.b * NC + c) * a.ld_src + m];
                        cur_b = e.b;
                    }
                    const double p = e.ux * x0 + e.uy * x1 + e.uz * x2;
                    const double r = p - rint(p);
                    float sn, cs;
                    sincospif(-2.0f * (float)r, &sn, &cs);
                    for (int c = 0; c < NC; c++) {
                        z[c].x = wl[c].x * cs - wl[c].y * sn;
                        z[c].y = wl[c].x * sn + wl[c].y * cs;
                    }
                }
#pragma unroll
                for (int p = 0; p < NF; p++) {
                    unsigned char *row = buf + (as * NF + p) * RS;
                    if constexpr (PREC == PB3) {
                        if constexpr (NX == 2) {
                            uint32_t h0, l0, h1, l1;
                            split2(z[2 * p].x, z[2 * p].y, h0, l0);
                            split2(z[2 * p + 1].x, z[2 * p + 1].y, h1, l1);
                            *(uint2 *)(row + msl * 8) = make_uint2(h0, h1);
                            *(uint2 *)(row + L::PLANEB + msl * 8) = make_uint2(l0, l1);
                        } else {
                            uint32_t h0, l0;
                            split2(z[p].x, z[p].y, h0, l0);
                            *(uint32_t *)(row + msl * 4) = h0;
                            *(uint32_t *)(row + L::PLANEB + msl * 4) = l0;
                        }
                    } else {
                        if constexpr (NX == 2)
                            *(float4 *)(row + msl * 16) = make_float4(z[2 * p].x, z[2 * p].y, z[2 * p + 1].x, z[2 * p + 1].y);
                        else
                            *(float2 *)(row + msl * 8) = z[p];
                    }
                }
            }
        };

        typedef f32x4 Acc;
        Acc acc_re[kTI][kTI], acc_im[kTI][kTI];
        for (int i = 0; i < kTI; i++)
            for (int j = 0; j < kTI; j++)
                for (int e = 0; e < 4; e++) {
                    acc_re[i][j][e] = 0.f;
                    acc_im[i][j][e] = 0.f;
                }
        const bool active = consumer && !(diag && wc > wr);
        const bool on_diag = diag && wc == wr;
        const int arow = wr * kWT;
        const int brow = (diag ? 0 : kST) + wc * kWT;

        auto consume = [&](const unsigned char *buf) {
            if constexpr (PREC == PB3) {
#pragma unroll
                for (int ks = 0; ks < kKC / 16; ks++) {
                    u32x4 ah[kTI], al[kTI], bh[kTI], bl[kTI];
#pragma unroll
                    for (int i = 0; i < kTI; i++) {
                        const unsigned char *p = buf + (arow + 16 * i + l16) * RS + ks * 64 + lk * 16;
                        ah[i] = *(const u32x4 *)p;
                        al[i] = *(const u32x4 *)(p + L::PLANEB);
                    }
#pragma unroll
                    for (int j = 0; j < kTI; j++) {
                        const unsigned char *p = buf + (brow + 16 * j + l16) * RS + ks * 64 + lk * 16;
                        bh[j] = *(const u32x4 *)p;
                        bl[j] = *(const u32x4 *)(p + L::PLANEB);
                    }
                    // per row tile: three passes over the column tiles, so updates of one
                    // accumulator are eight MFMAs apart
#pragma unroll
                    for (int i = 0; i < kTI; i++) {
                        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[i]);
                        const bf16x8 Al = __builtin_bit_cast(bf16x8, al[i]);
                        const bf16x8 Wh = __builtin_bit_cast(bf16x8, bf16_rot(ah[i]));
                        const bf16x8 Wl = __builtin_bit_cast(bf16x8, bf16_rot(al[i]));
#pragma unroll
                        for (int j = 0; j < kTI; j++) {
                            const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]);
                            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc_re[i][j], 0, 0, 0);
                            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wh, Bh, acc_im[i][j], 0, 0, 0);
                        }
#pragma unroll
                        for (int j = 0; j < kTI; j++) {
                            const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[j]);
                            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc_re[i][j], 0, 0, 0);
                            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wh, Bl, acc_im[i][j], 0, 0, 0);
                        }
#pragma unroll
                        for (int j = 0; j < kTI; j++) {
                            const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]);
                            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc_re[i][j], 0, 0, 0);
                            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl, Bh, acc_im[i][j], 0, 0, 0);
                        }
                        // lo lo^H only where it is a one-signed bias: the output diagonal
                        if (on_diag) {
                            const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[i]);
                            acc_re[i][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bl, acc_re[i][i], 0, 0, 0);
                            acc_im[i][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl, Bl, acc_im[i][i], 0, 0, 0);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < kKC; kk += 4) {
                    float2 av[kTI], bv[kTI];
#pragma unroll
                    for (int i = 0; i < kTI; i++) av[i] = *(const float2 *)(buf + (arow + 16 * i + l16) * RS + (kk + lk) * 8);
#pragma unroll
                    for (int j = 0; j < kTI; j++) bv[j] = *(const float2 *)(buf + (brow + 16 * j + l16) * RS + (kk + lk) * 8);
#pragma unroll
                    for (int i = 0; i < kTI; i++) {
                        const float nre = -av[i].x;
#pragma unroll
                        for (int j = 0; j < kTI; j++) {
                            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, acc_re[i][j], 0, 0, 0);
                            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].x, acc_im[i][j], 0, 0, 0);
                        }
#pragma unroll
                        for (int j = 0; j < kTI; j++) {
                            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, acc_re[i][j], 0, 0, 0);
                            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nre, bv[j].y, acc_im[i][j], 0, 0, 0);
                        }
                    }
                }
            }
        };

        if (!consumer) fetch(0);
        __syncthreads();  // antenna table ready
        if (!consumer) {
            produce(lds);
            fetch(1);
        }
        __syncthreads();
        for (int stg = 0; stg < n_stage; stg++) {
            unsigned char *cur = lds + (stg & 1) * L::BUF;
            unsigned char *nxt = lds + ((stg + 1) & 1) * L::BUF;
            if (consumer) {
                if (active) consume(cur);
            } else if (stg + 1 < n_stage) {
                produce(nxt);
                fetch(stg + 2);
            }
            __syncthreads();
        }

        if (active) {
            float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
            const int rb = I * kST + wr * kWT + 4 * lk;
            const int c0 = J * kST + wc * kWT + l16;
#pragma unroll
            for (int i = 0; i < kTI; i++)
#pragma unroll
                for (int j = 0; j < kTI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        P[(int64_t)(rb + 16 * i + e) * Np + c0 + 16 * j] = make_float2(acc_re[i][j][e], acc_im[i][j][e]);
        }
    }
}

template <int PREC>
hipError_t launch_prec(const FusedArgs &a, hipStream_t s) {
    if (a.n_feed == 2 && a.n_ax == 2)
        k_herk_fused<PREC, 2, 2><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_feed == 2)
        k_herk_fused<PREC, 2, 1><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_ax == 2)
        k_herk_fused<PREC, 1, 2><<<a.grid, 512, 0, s>>>(a);
    else
        k_herk_fused<PREC, 1, 1><<<a.grid, 512, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_herk_fused(int prec, const FusedArgs &a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    if (prec == P32) return launch_prec<P32>(a, s);
    if (prec == PB3) return launch_prec<PB3>(a, s);
    return hipErrorInvalidValue;
}

int herk_fused_occupancy(int prec) {
    int nb = 1;
    hipError_t e = prec == P32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk_fused<P32, 2, 2>, 512, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk_fused<PB3, 2, 2>, 512, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb < 1 ? 1 : nb;
}

}  // namespace mv
