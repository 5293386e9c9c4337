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
// on BF16X3); the consumers form the last rows of each stage after their
// products.  One barrier per stage swaps the buffers, so the VALU work of
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
#include "matvis.h"
#include "internal.h"
#include <type_traits>

namespace mv {

namespace {

constexpr int kST = 128, kWT = 64, kKC = 32, kTI = 4;

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Row of a forming thread (8 threads per row, two sources each): a wave's 8 rows
// in the order 0, 4, 1, 5, 2, 6, 3, 7, so the two rows that 16 consecutive
// lanes write are 4 rows (576 bytes) apart and fall in disjoint LDS banks.
__device__ inline int wrow(int t) {
    const int g = (t >> 3) & 7;
    return ((t >> 6) << 3) + (((g & 1) << 2) | (g >> 1));
}

// The same for 160-byte rows: rows 0, 2, 1, 3, 4, 6, 5, 7 (two rows 320 bytes, 16
// banks, apart)
__device__ inline int wrow160(int t) {
    const int g = (t >> 3) & 7;
    return ((t >> 6) << 3) + (g & 4) + ((g & 1) << 1) + ((g >> 1) & 1);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// packed (hi, lo) bf16 words of one complex64 value: hi = bf16(z), lo = bf16(z - hi),
// both round-to-nearest-even (v_cvt_pk_bf16_f32 on gfx950)
__device__ inline void split2(float re, float im, uint32_t &hi, uint32_t &lo) {
    const f32x2_t z = {re, im};
    const bf16x2_t h = __builtin_convertvector(z, bf16x2_t);
    const f32x2_t r = z - __builtin_convertvector(h, f32x2_t);
    const bf16x2_t l = __builtin_convertvector(r, bf16x2_t);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
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

// ---------------------------------------------------------------------------
// Consumers.  An accumulator pair (re, im) per 16 x 16 output tile; one
// k-stage (KC = 32 complex columns) is read from the LDS stage buffer, whose
// rows 0..127 hold block I and rows 128..255 block J.
//
// BF16X3 tile update with row operand (Ah, Al, Wh, Wl) and column operand
// (Bh, Bl): re += Ah Bh + Ah Bl + Al Bh, im += Wh Bh + Wh Bl + Wl Bh, and on
// output-diagonal tiles also the lo lo products (a one-signed |lo|^2 bias
// there; elsewhere it averages out and is omitted).
// FP32 tile update with one complex element per lane (a, b):
// re += a.re b.re + a.im b.im, im += a.im b.re - a.re b.im.
// ---------------------------------------------------------------------------

struct RowB3 {
    bf16x8 h, l, wh, wl;
};

template <int PREC>
__device__ __forceinline__ RowB3 load_row_b3(const unsigned char *buf, int row, int ks, int lk) {
    typedef FL<PREC> L;
    const unsigned char *p = buf + row * L::RS + ks * 64 + lk * 16;
    const u32x4 h = *(const u32x4 *)p;
    const u32x4 l = *(const u32x4 *)(p + L::PLANEB);
    RowB3 r;
    r.h = __builtin_bit_cast(bf16x8, h);
    r.l = __builtin_bit_cast(bf16x8, l);
    r.wh = __builtin_bit_cast(bf16x8, bf16_rot(h));
    r.wl = __builtin_bit_cast(bf16x8, bf16_rot(l));
    return r;
}

// Off-diagonal super-tile: wave tile of 4 x 4 tiles (rows arow.., columns brow..).
template <int PREC>
__device__ __forceinline__ void consume_full(const unsigned char *buf, int arow, int brow, int l16, int lk,
                                             f32x4 (&re)[16], f32x4 (&im)[16]) {
    typedef FL<PREC> L;
    if constexpr (PREC == PB3) {
#pragma unroll
        for (int ks = 0; ks < kKC / 16; ks++) {
            RowB3 A[kTI];
#pragma unroll
            for (int i = 0; i < kTI; i++) A[i] = load_row_b3<PREC>(buf, arow + 16 * i + l16, ks, lk);
            const unsigned char *pc = buf + (brow + l16) * L::RS + ks * 64 + lk * 16;
            u32x4 nh = *(const u32x4 *)pc, nl = *(const u32x4 *)(pc + L::PLANEB);
#pragma unroll
            for (int j = 0; j < kTI; j++) {
                const bf16x8 Bh = __builtin_bit_cast(bf16x8, nh);
                const bf16x8 Bl = __builtin_bit_cast(bf16x8, nl);
                if (j + 1 < kTI) {
                    const unsigned char *p = pc + 16 * (j + 1) * L::RS;
                    nh = *(const u32x4 *)p;
                    nl = *(const u32x4 *)(p + L::PLANEB);
                }
#pragma unroll
                for (int i = 0; i < kTI; i++) {
                    re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].h, Bh, re[i * kTI + j], 0, 0, 0);
                    im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].wh, Bh, im[i * kTI + j], 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < kTI; i++) {
                    re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].h, Bl, re[i * kTI + j], 0, 0, 0);
                    im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].wh, Bl, im[i * kTI + j], 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < kTI; i++) {
                    re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].l, Bh, re[i * kTI + j], 0, 0, 0);
                    im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i].wl, Bh, im[i * kTI + j], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            float2 av[kTI], bv[kTI];
#pragma unroll
            for (int i = 0; i < kTI; i++) av[i] = *(const float2 *)(buf + (arow + 16 * i + l16) * L::RS + (kk + lk) * 8);
#pragma unroll
            for (int j = 0; j < kTI; j++) bv[j] = *(const float2 *)(buf + (brow + 16 * j + l16) * L::RS + (kk + lk) * 8);
#pragma unroll
            for (int i = 0; i < kTI; i++) {
                const float nre = -av[i].x;
#pragma unroll
                for (int j = 0; j < kTI; j++) {
                    re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, re[i * kTI + j], 0, 0, 0);
                    im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].x, im[i * kTI + j], 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < kTI; j++) {
                    re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, re[i * kTI + j], 0, 0, 0);
                    im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nre, bv[j].y, im[i * kTI + j], 0, 0, 0);
                }
            }
        }
    }
}

// Diagonal super-tile: its lower triangle has 36 tiles; wave W takes the
// 16-row blocks W and 7 - W, i.e. tiles (7 - W, 0..7 - W) in slots
// 0..7 - W and (W, 0..W) in slots 8 - W.., nine tiles for every wave.
template <int PREC, int W>
__device__ __forceinline__ void consume_tri(const unsigned char *buf, int l16, int lk, f32x4 (&re)[16],
                                            f32x4 (&im)[16]) {
    typedef FL<PREC> L;
    constexpr int R1 = 7 - W, R0 = W, NCOL = 8 - W;
    if constexpr (PREC == PB3) {
#pragma unroll
        for (int ks = 0; ks < kKC / 16; ks++) {
            const RowB3 a1 = load_row_b3<PREC>(buf, 16 * R1 + l16, ks, lk);
            const RowB3 a0 = load_row_b3<PREC>(buf, 16 * R0 + l16, ks, lk);
            // column fragments are prefetched one tile ahead; the scheduling fences
            // keep the compiler from hoisting every column's loads (register pressure)
            const unsigned char *pc = buf + l16 * L::RS + ks * 64 + lk * 16;
            u32x4 nh = *(const u32x4 *)pc, nl = *(const u32x4 *)(pc + L::PLANEB);
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                const bf16x8 Bh = __builtin_bit_cast(bf16x8, nh);
                const bf16x8 Bl = __builtin_bit_cast(bf16x8, nl);
                if (c + 1 < NCOL) {
                    const unsigned char *p = pc + 16 * (c + 1) * L::RS;
                    nh = *(const u32x4 *)p;
                    nl = *(const u32x4 *)(p + L::PLANEB);
                }
                const int s1 = c, s0 = NCOL + c;
                const bool two = c <= R0;
                re[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.h, Bh, re[s1], 0, 0, 0);
                im[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.wh, Bh, im[s1], 0, 0, 0);
                if (two) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.h, Bh, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.wh, Bh, im[s0], 0, 0, 0);
                }
                re[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.h, Bl, re[s1], 0, 0, 0);
                im[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.wh, Bl, im[s1], 0, 0, 0);
                if (two) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.h, Bl, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.wh, Bl, im[s0], 0, 0, 0);
                }
                re[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.l, Bh, re[s1], 0, 0, 0);
                im[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.wl, Bh, im[s1], 0, 0, 0);
                if (two) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.l, Bh, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.wl, Bh, im[s0], 0, 0, 0);
                }
                if (c == R1) {
                    re[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.l, Bl, re[s1], 0, 0, 0);
                    im[s1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.wl, Bl, im[s1], 0, 0, 0);
                }
                if (c == R0) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.l, Bl, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.wl, Bl, im[s0], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            const float2 a1 = *(const float2 *)(buf + (16 * R1 + l16) * L::RS + (kk + lk) * 8);
            const float2 a0 = *(const float2 *)(buf + (16 * R0 + l16) * L::RS + (kk + lk) * 8);
            const float n1 = -a1.x, n0 = -a0.x;
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                const float2 b = *(const float2 *)(buf + (16 * c + l16) * L::RS + (kk + lk) * 8);
                const int s1 = c, s0 = NCOL + c;
                re[s1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, b.x, re[s1], 0, 0, 0);
                im[s1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, b.x, im[s1], 0, 0, 0);
                if (c <= R0) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, b.x, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, b.x, im[s0], 0, 0, 0);
                }
                re[s1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, b.y, re[s1], 0, 0, 0);
                im[s1] = __builtin_amdgcn_mfma_f32_16x16x4f32(n1, b.y, im[s1], 0, 0, 0);
                if (c <= R0) {
                    re[s0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, b.y, re[s0], 0, 0, 0);
                    im[s0] = __builtin_amdgcn_mfma_f32_16x16x4f32(n0, b.y, im[s0], 0, 0, 0);
                }
            }
        }
    }
}

// One launch per item kind: DIAG = the nb diagonal super-tiles (I, I) of each
// (instance, k-split), consumed with the triangular wave mapping; otherwise the
// nb (nb - 1) / 2 off-diagonal ones (I > J), consumed as 2 x 2 wave tiles.
// a.work is the per-instance prefix of k-splits; instance i owns items
// [work[i] n_kind, work[i + 1] n_kind).
template <int PREC, int NF, int NX, bool DIAG>
__global__ void __launch_bounds__(512, 1) k_herk_fused(FusedArgs a) {
    typedef FL<PREC> L;
    constexpr int RS = L::RS;
    constexpr int NC = NF * NX;       // beam components per source
    constexpr int SPS = kKC / NX;     // sources per stage
    constexpr int APB = kST / NF;     // antennas per row block
    constexpr int NG = 256 / SPS;     // thread groups per wave kind (one source per thread)
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
    const int n_kind = DIAG ? nb : nb * (nb - 1) / 2;
    const int total = a.work[a.n_inst] * n_kind;
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    // forming roles: source msl of the stage; group g of the thread's wave kind
    const int msl = tid % SPS, g = (tid % 256) / SPS;
    constexpr bool diag = DIAG;

    for (int item = slot_x; item < total; item += a.grid) {
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work[mid] * n_kind <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int inst = lo;
        const int local = item - a.work[inst] * n_kind;
        const int s = local / n_kind;
        int st = local % n_kind;
        int I, J;
        if (DIAG) {
            I = J = st;
        } else {  // st enumerates the pairs (1, 0), (2, 0), (2, 1), (3, 0), ...
            I = 1;
            while (st >= I) {
                st -= I;
                I++;
            }
            J = st;
        }
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.kcols[inst] / NX;
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

        // direction and beam of this thread's source in the next stage
        double sx = 0.0, sy = 0.0, sz = 0.0;
        float2 w[NC];
        bool live = false;
        int64_t m_cur = 0;
        auto fetch = [&](int stage) {
            m_cur = m_begin + (int64_t)stage * SPS + msl;
            live = stage < n_stage && m_cur < m_end;
            sx = sy = sz = 0.0;
            for (int c = 0; c < NC; c++) w[c] = make_float2(0.f, 0.f);
            if (live) {
                sx = sh[m_cur];
                sy = sh[a.ld_src + m_cur];
                sz = sh[2 * a.ld_src + m_cur];
                if (a.n_beam == 1)
                    for (int c = 0; c < NC; c++) w[c] = Bm[(int64_t)c * a.ld_src + m_cur];
            }
        };

        // ---- producer: form the Z rows of blocks I (and J) for one stage.
        // The fringe factor uses the hardware sine / cosine, whose argument is in
        // revolutions, on the FP64-reduced phase r in [-1/2, 1/2]:
        // F = exp(-2 pi i r) = cos(-r rev) + i sin(-r rev).  Rows past n_ant and
        // sources past the split are written as zeros (mask factor 0).
        // The consumers form the last rows of each stage after their products (an
        // off-diagonal item's rows: 3/8 with one beam component, whose rows are
        // cheap to form, else 1/4; half that on a diagonal item, where the products
        // are fewer); the producers form the rest.
        const int n_crow = (NC == 1 ? 3 * na_tot / 8 : na_tot / 4) / (diag ? 2 : 1);
        const int row0 = consumer ? na_tot - n_crow : 0, row1 = consumer ? na_tot : na_tot - n_crow;
        auto produce = [&](unsigned char *buf) {
            const bool lv = live;
            const double x0 = sx, x1 = sy, x2 = sz;
            const int64_t m = m_cur;
            float2 wl[NC];
            for (int c = 0; c < NC; c++) wl[c] = w[c];
            const bool multi_beam = a.n_beam != 1;
            int cur_b = multi_beam ? -1 : 0;
            for (int as = row0 + g; as < row1; as += NG) {
                const AntEntry e = tab[as];
                if (multi_beam && lv && e.b >= 0 && e.b != cur_b) {
                    for (int c = 0; c < NC; c++) wl[c] = Bm[((int64_t)e.b * NC + c) * a.ld_src + m];
                    cur_b = e.b;
                }
                const double p = e.ux * x0 + e.uy * x1 + e.uz * x2;
                const float r = (float)(p - rint(p));
                const float msk = (lv && e.b >= 0) ? 1.0f : 0.0f;
                const float sn = msk * __builtin_amdgcn_sinf(-r);
                const float cs = msk * __builtin_amdgcn_cosf(-r);
                float2 z[NC];
                for (int c = 0; c < NC; c++) {
                    z[c].x = wl[c].x * cs - wl[c].y * sn;
                    z[c].y = wl[c].x * sn + wl[c].y * cs;
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

        f32x4 acc_re[16], acc_im[16];
        for (int t = 0; t < 16; t++)
            for (int e = 0; e < 4; e++) {
                acc_re[t][e] = 0.f;
                acc_im[t][e] = 0.f;
            }
        const int arow = wr * kWT;
        const int brow = kST + wc * kWT;

        auto consume = [&](const unsigned char *buf) {
            if constexpr (!DIAG) {
                consume_full<PREC>(buf, arow, brow, l16, lk, acc_re, acc_im);
            } else {
                switch (wave) {
                    case 0: consume_tri<PREC, 0>(buf, l16, lk, acc_re, acc_im); break;
                    case 1: consume_tri<PREC, 1>(buf, l16, lk, acc_re, acc_im); break;
                    case 2: consume_tri<PREC, 2>(buf, l16, lk, acc_re, acc_im); break;
                    default: consume_tri<PREC, 3>(buf, l16, lk, acc_re, acc_im); break;
                }
            }
        };

        fetch(0);
        __syncthreads();  // antenna table ready
        produce(lds);
        fetch(1);
        __syncthreads();
        for (int stg = 0; stg < n_stage; stg++) {
            unsigned char *cur = lds + (stg & 1) * L::BUF;
            unsigned char *nxt = lds + ((stg + 1) & 1) * L::BUF;
            if (consumer) consume(cur);
            if (stg + 1 < n_stage) {
                produce(nxt);
                fetch(stg + 2);
            }
            __syncthreads();
        }

        if (consumer) {
            float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
            if constexpr (!DIAG) {
                const int rb = I * kST + wr * kWT + 4 * lk;
                const int c0 = J * kST + wc * kWT + l16;
#pragma unroll
                for (int i = 0; i < kTI; i++)
#pragma unroll
                    for (int j = 0; j < kTI; j++)
#pragma unroll
                        for (int e = 0; e < 4; e++)
                            P[(int64_t)(rb + 16 * i + e) * Np + c0 + 16 * j] =
                                make_float2(acc_re[i * kTI + j][e], acc_im[i * kTI + j][e]);
            } else {
                // slot t of wave w: tile (7 - w, t) for t < 8 - w, else tile (w, t - (8 - w))
                const int ncol = 8 - wave;
#pragma unroll
                for (int t = 0; t < 9; t++) {
                    const int R = t < ncol ? 7 - wave : wave;
                    const int C = t < ncol ? t : t - ncol;
                    const int r0 = I * kST + 16 * R + 4 * lk;
                    const int c0 = I * kST + 16 * C + l16;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        P[(int64_t)(r0 + e) * Np + c0] = make_float2(acc_re[t][e], acc_im[t][e]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two-block items (BF16X3, 129..256 rows): one workgroup owns every row of an
// (instance, k-split), so each Z element is formed exactly once, and all
// eight waves both form Z and run MFMA products.  The 136 lower-triangle
// 16 x 16 tiles of the 256 x 256 product are split as
//   waves 0-3: the off-diagonal 128 x 128 block, a 64 x 64 wave tile each;
//   waves 4-7: the two 128-row diagonal triangles, rows {0, 7, 1, 6} or
//              {2, 5, 3, 4} of one triangle (18 tiles each).
// Waves w and w + 4 share a SIMD; the first forms Z after its products and
// the second before them, so matrix and vector work overlap on every SIMD.
// The column operand carries the rotation here: im += a . (-b_im, b_re).
// ---------------------------------------------------------------------------

// the column fragment rotated for the imaginary part: (re, im) -> (-im, re) per bf16 pair
__device__ inline u32x4 bf16_rot_col(u32x4 v) {
    u32x4 r;
    for (int q = 0; q < 4; q++) r[q] = __builtin_amdgcn_alignbit(v[q], v[q], 16) ^ 0x00008000u;
    return r;
}

__device__ __forceinline__ void mfma_pair(const u32x4 &a, const u32x4 &b, const u32x4 &w, f32x4 &re, f32x4 &im) {
    re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), re, 0, 0,
                                                 0);
    im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, w), im, 0, 0,
                                                 0);
}

// Staged-row geometry of the two-block kernels: RS bytes per row, hi plane
// then lo plane of PLANEB bytes each, NKS k-steps of 16 complex per stage.
// Operand reads are 16 bytes per lane from 16 rows at once; measured on the
// LDS, 160-byte rows serve them without bank conflicts and 144-byte rows with
// half of their cycles in conflicts, so 160 bytes where the stage buffers fit.
template <int RS_, int PLANEB_, int NKS_>
struct RowGeom {
    static constexpr int RS = RS_, PLANEB = PLANEB_, NKS = NKS_;
};
typedef RowGeom<FL<PB3>::RS, FL<PB3>::PLANEB, kKC / 16> GeomPair;  // 32 complex per stage
typedef RowGeom<16 * 4 * 2 + 16, 16 * 4, 1> GeomCoh;               // 16 complex per stage
typedef RowGeom<16 * 4 * 2 + 32, 16 * 4, 1> GeomCoh3;              // the same in 160-byte rows
typedef RowGeom<FL<PB3>::RS + 16, FL<PB3>::PLANEB, kKC / 16> GeomPair3;  // 32 complex, 288-byte rows

// Off-diagonal block: rows 16 (rb + i), columns 16 (cb + j), i < NR, j < NC
// (4 x 4 tiles, or 3 x 3 on a short diagonal block); tile (i, j) accumulates
// in slot i * kTI + j.
template <typename L, int NACC, int NR = kTI, int NC = kTI>
__device__ __forceinline__ void consume_sq_b3(const unsigned char *buf, int rb, int cb, int l16, int lk,
                                              f32x4 (&re)[NACC], f32x4 (&im)[NACC]) {
#pragma unroll
    for (int ks = 0; ks < L::NKS; ks++) {
        // loads in the order of first use: hi rows, the first column, lo rows
        u32x4 ah[NR], al[NR];
#pragma unroll
        for (int i = 0; i < NR; i++) ah[i] = *(const u32x4 *)(buf + (16 * (rb + i) + l16) * L::RS + ks * 64 + lk * 16);
        const unsigned char *pc = buf + (16 * cb + l16) * L::RS + ks * 64 + lk * 16;
        u32x4 nh = *(const u32x4 *)pc, nl = *(const u32x4 *)(pc + L::PLANEB);
#pragma unroll
        for (int i = 0; i < NR; i++)
            al[i] = *(const u32x4 *)(buf + (16 * (rb + i) + l16) * L::RS + ks * 64 + lk * 16 + L::PLANEB);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < NC; j++) {
            const u32x4 bh = nh, bl = nl;
            if (j + 1 < NC) {
                const unsigned char *p = pc + 16 * (j + 1) * L::RS;
                nh = *(const u32x4 *)p;
                nl = *(const u32x4 *)(p + L::PLANEB);
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this column's products
            const u32x4 wh = bf16_rot_col(bh), wl = bf16_rot_col(bl);
            // one product term for every row before the next, so that MFMAs into the
            // same accumulator are 2 NR issues apart
#pragma unroll
            for (int i = 0; i < NR; i++) mfma_pair(ah[i], bh, wh, re[i * kTI + j], im[i * kTI + j]);
#pragma unroll
            for (int i = 0; i < NR; i++) mfma_pair(ah[i], bl, wl, re[i * kTI + j], im[i * kTI + j]);
#pragma unroll
            for (int i = 0; i < NR; i++) mfma_pair(al[i], bh, wh, re[i * kTI + j], im[i * kTI + j]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Row sets of the triangle waves and the first accumulator slot of each row
// (row r of a set holds columns 0..r in consecutive slots).  On a diagonal
// block the column operand of column c is the row operand of row c (same
// rows, same lane layout), so a wave loads only the columns that are not its
// own rows, and none right of its last row.  order[] interleaves loaded and
// reused columns so every load has at least one column of products to hide in.
template <int S>
struct TriSet {
    static constexpr int NR = 4;
    static constexpr int r[4] = {S == 0 ? 0 : 2, S == 0 ? 7 : 5, S == 0 ? 1 : 3, S == 0 ? 6 : 4};
    static constexpr int base[4] = {0, r[0] + 1, r[0] + r[1] + 2, r[0] + r[1] + r[2] + 3};
    static constexpr int ncol = S == 0 ? 8 : 6;
    static constexpr int order[8] = {S == 0 ? 0 : 2, S == 0 ? 2 : 0, S == 0 ? 1 : 3, S == 0 ? 3 : 1,
                                     S == 0 ? 6 : 4, S == 0 ? 4 : 5, S == 0 ? 7 : -1, S == 0 ? 5 : -1};
    // row slot holding column c, or -1 when the column is loaded
    static constexpr int slot(int c) { return r[0] == c ? 0 : r[1] == c ? 1 : r[2] == c ? 2 : r[3] == c ? 3 : -1; }
    // first position at or after p whose column is loaded, or -1
    static constexpr int next_loaded(int p) {
        return p >= ncol ? -1 : slot(order[p]) < 0 ? p : next_loaded(p + 1);
    }
};

// Two-row sets {S, 7 - S} of a 128-row triangle (nine tiles each), columns in
// natural order; rows S and 7 - S double as columns S and 7 - S.
template <int S>
struct TriPair {
    static constexpr int NR = 2;
    static constexpr int r[2] = {S, 7 - S};
    static constexpr int base[2] = {0, S + 1};
    static constexpr int ncol = 8 - S;
    static constexpr int order[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    static constexpr int slot(int c) { return c == r[0] ? 0 : c == r[1] ? 1 : -1; }
    static constexpr int next_loaded(int p) {
        return p >= ncol ? -1 : slot(order[p]) < 0 ? p : next_loaded(p + 1);
    }
};

// A tile set passed as a value (to pick a set at run time among instantiations)
template <typename T>
struct SetTag {
    typedef T type;
};

// Row S alone of a two-row set, when row 7 - S lies wholly past the antennas of
// a short last block (its tiles are neither multiplied nor stored).
template <int S>
struct TriSingle {
    static constexpr int NR = 1;
    static constexpr int r[1] = {S};
    static constexpr int base[1] = {0};
    static constexpr int ncol = S + 1;
    static constexpr int order[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    static constexpr int slot(int c) { return c == r[0] ? 0 : -1; }
    static constexpr int next_loaded(int p) {
        return p >= ncol ? -1 : slot(order[p]) < 0 ? p : next_loaded(p + 1);
    }
};

// Row sets of the triangle waves on a short diagonal block of at most 96
// antennas (six tile rows): {5, 0, 3} (eleven tiles) and {4, 1, 2} (ten).
template <int S>
struct TriSet6 {
    static constexpr int NR = 3;
    static constexpr int r[3] = {S == 0 ? 5 : 4, S == 0 ? 0 : 1, S == 0 ? 3 : 2};
    static constexpr int base[3] = {0, r[0] + 1, r[0] + r[1] + 2};
    static constexpr int ncol = S == 0 ? 6 : 5;
    static constexpr int order[6] = {S == 0 ? 0 : 1, S == 0 ? 1 : 0, S == 0 ? 3 : 2,
                                     S == 0 ? 2 : 3, S == 0 ? 5 : 4, S == 0 ? 4 : -1};
    static constexpr int slot(int c) { return r[0] == c ? 0 : r[1] == c ? 1 : r[2] == c ? 2 : -1; }
    static constexpr int next_loaded(int p) {
        return p >= ncol ? -1 : slot(order[p]) < 0 ? p : next_loaded(p + 1);
    }
};

// Calls f(slot, row, column) for every tile of a triangle row set.
template <typename T, typename F>
__device__ __forceinline__ void for_tri_tiles(F f) {
#pragma unroll
    for (int k = 0; k < T::NR; k++)
#pragma unroll
        for (int c = 0; c <= T::r[k]; c++) f(T::base[k] + c, T::r[k], c);
}

// One 128-row diagonal triangle starting at LDS row o: tiles (r, c), c <= r, r in the set.
template <typename L, typename T, int NACC>
__device__ __forceinline__ void consume_tri_b3(const unsigned char *buf, int o, int l16, int lk, f32x4 (&re)[NACC],
                                               f32x4 (&im)[NACC]) {
    constexpr int NR = T::NR;
#pragma unroll
    for (int ks = 0; ks < L::NKS; ks++) {
        const unsigned char *p0 = buf + (o + l16) * L::RS + ks * 64 + lk * 16;  // row / column 0 of this lane
        u32x4 ah[NR], al[NR];
#pragma unroll
        for (int k = 0; k < NR; k++) {
            ah[k] = *(const u32x4 *)(p0 + 16 * T::r[k] * L::RS);
            al[k] = *(const u32x4 *)(p0 + 16 * T::r[k] * L::RS + L::PLANEB);
        }
        u32x4 nh = {0u, 0u, 0u, 0u}, nl = {0u, 0u, 0u, 0u};
        constexpr int f0 = T::next_loaded(0);
        if (f0 >= 0) {
            nh = *(const u32x4 *)(p0 + 16 * T::order[f0] * L::RS);
            nl = *(const u32x4 *)(p0 + 16 * T::order[f0] * L::RS + L::PLANEB);
        }
#pragma unroll
        for (int q = 0; q < T::ncol; q++) {
            const int c = T::order[q];
            const int kc = T::slot(c);
            u32x4 bh, bl;
            if (kc >= 0) {
                bh = ah[kc];
                bl = al[kc];
            } else {
                bh = nh;
                bl = nl;
                const int qn = T::next_loaded(q + 1);
                if (qn >= 0) {
                    nh = *(const u32x4 *)(p0 + 16 * T::order[qn] * L::RS);
                    nl = *(const u32x4 *)(p0 + 16 * T::order[qn] * L::RS + L::PLANEB);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            const u32x4 wh = bf16_rot_col(bh), wl = bf16_rot_col(bl);
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (T::r[k] >= c) mfma_pair(ah[k], bh, wh, re[T::base[k] + c], im[T::base[k] + c]);
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (T::r[k] >= c) mfma_pair(ah[k], bl, wl, re[T::base[k] + c], im[T::base[k] + c]);
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (T::r[k] >= c) mfma_pair(al[k], bh, wh, re[T::base[k] + c], im[T::base[k] + c]);
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (T::r[k] == c) mfma_pair(al[k], bl, wl, re[T::base[k] + c], im[T::base[k] + c]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// FP32 forms of the two wave shapes on a stage of 16 complex columns (one
// complex64 per element, re/im interleaved): per 4-deep k group,
// re += a.re b.re + a.im b.im and im += a.im b.re - a.re b.im on
// v_mfma_f32_16x16x4f32, one complex element per lane.
template <typename L, int NACC, int NR = kTI, int NC = kTI>
__device__ __forceinline__ void consume_sq_f32(const unsigned char *buf, int rb, int cb, int l16, int lk,
                                               f32x4 (&re)[NACC], f32x4 (&im)[NACC]) {
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
        float2 av[NR], bv[NC];
#pragma unroll
        for (int i = 0; i < NR; i++) av[i] = *(const float2 *)(buf + (16 * (rb + i) + l16) * L::RS + (kk + lk) * 8);
#pragma unroll
        for (int j = 0; j < NC; j++) bv[j] = *(const float2 *)(buf + (16 * (cb + j) + l16) * L::RS + (kk + lk) * 8);
#pragma unroll
        for (int i = 0; i < NR; i++) {
            const float nre = -av[i].x;
#pragma unroll
            for (int j = 0; j < NC; j++) {
                re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, re[i * kTI + j], 0, 0, 0);
                im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].x, im[i * kTI + j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < NC; j++) {
                re[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, re[i * kTI + j], 0, 0, 0);
                im[i * kTI + j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nre, bv[j].y, im[i * kTI + j], 0, 0, 0);
            }
        }
    }
}

template <typename L, typename T, int NACC>
__device__ __forceinline__ void consume_tri_f32(const unsigned char *buf, int o, int l16, int lk, f32x4 (&re)[NACC],
                                                f32x4 (&im)[NACC]) {
    constexpr int NR = T::NR;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
        const unsigned char *p0 = buf + (o + l16) * L::RS + (kk + lk) * 8;
        float2 av[NR];
#pragma unroll
        for (int k = 0; k < NR; k++) av[k] = *(const float2 *)(p0 + 16 * T::r[k] * L::RS);
#pragma unroll
        for (int q = 0; q < T::ncol; q++) {
            const int c = T::order[q];
            const int kc = T::slot(c);
            // a column that is one of the wave's rows is already in registers
            const float2 b = kc >= 0 ? av[kc] : *(const float2 *)(p0 + 16 * c * L::RS);
#pragma unroll
            for (int k = 0; k < NR; k++)
                if (T::r[k] >= c) {
                    f32x4 &r = re[T::base[k] + c], &m = im[T::base[k] + c];
                    r = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k].x, b.x, r, 0, 0, 0);
                    m = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k].y, b.x, m, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k].y, b.y, r, 0, 0, 0);
                    m = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[k].x, b.y, m, 0, 0, 0);
                }
        }
    }
}

template <int NC>
struct SrcEntry {
    double x, y, z;   // s_hat of the source
    float2 w[NC];     // its beam values (one unique beam)
    int64_t m;        // source index, -1 past the split
};

template <int NF, int NX>
__global__ void __launch_bounds__(512, 1) k_herk_b3_pair(FusedArgs a) {
    typedef FL<PB3> L;
    constexpr int RS = L::RS;
    constexpr int NC = NF * NX;       // beam components per source
    constexpr int SPS = kKC / NX;     // sources per stage
    constexpr int NA = 2 * kST / NF;  // antennas of the 256 rows
    constexpr int NG = 512 / SPS;     // thread groups (one source per thread)
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * L::BUF];
    __shared__ AntEntry tab[NA];
    __shared__ SrcEntry<NC> src[2][SPS];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const bool sq = wave < 4;
    const int l16 = lane & 15, lk = lane >> 4;
    const int Np = a.n_rows_pad;  // 256
    const int total = a.work[a.n_inst];
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int msl = tid % SPS, g = tid / SPS;
    // wave roles: square tile origin, or triangle (row offset, row set)
    const int sq_rb = 8 + 4 * (wave >> 1), sq_cb = 4 * (wave & 1);
    const int tri_o = ((wave - 4) >> 1) * kST, tri_s = (wave - 4) & 1;

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
        const int s = item - a.work[inst];
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.kcols[inst] / NX;
        const int64_t m_begin = (int64_t)s * ms_per_split;
        const int64_t m_end = m_begin + ms_per_split < M ? m_begin + ms_per_split : M;
        const int n_stage = (int)((m_end - m_begin + SPS - 1) / SPS);
        const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
        const float2 *Bm = (const float2 *)a.B + (int64_t)inst * a.n_beam * NC * a.ld_src;

        {
            const double nu_c = a.freqs[f] / kSpeedOfLight;
            for (int as = tid; as < NA; as += 512) {
                AntEntry e;
                if (as < a.n_ant) {
                    e.ux = nu_c * a.antc[3 * as];
                    e.uy = nu_c * a.antc[3 * as + 1];
                    e.uz = nu_c * a.antc[3 * as + 2];
                    e.b = a.bidx[as];
                } else {
                    e.ux = e.uy = e.uz = 0.0;
                    e.b = -1;
                }
                e.pad = 0;
                tab[as] = e;
            }
        }

        // Source data of a stage (direction, beam, index) is loaded by the first
        // SPS lanes of wave 0 one stage ahead and kept in LDS (src[stage & 1]),
        // so no other wave holds it in registers while it runs its products.
        double fx = 0.0, fy = 0.0, fz = 0.0;
        float2 fw[NC];
        int64_t fm = -1;
        const bool fetcher = tid < SPS;
        auto fetch = [&](int stage) {  // issue the loads (wave 0)
            const int64_t m = m_begin + (int64_t)stage * SPS + tid;
            fm = (stage < n_stage && m < m_end) ? m : -1;
            fx = fy = fz = 0.0;
            for (int c = 0; c < NC; c++) fw[c] = make_float2(0.f, 0.f);
            if (fm >= 0) {
                fx = sh[fm];
                fy = sh[a.ld_src + fm];
                fz = sh[2 * a.ld_src + fm];
                if (a.n_beam == 1)
                    for (int c = 0; c < NC; c++) fw[c] = Bm[(int64_t)c * a.ld_src + fm];
            }
        };
        auto stash = [&](int stage) {  // publish them (wave 0)
            SrcEntry<NC> &e = src[stage & 1][tid];
            e.x = fx;
            e.y = fy;
            e.z = fz;
            for (int c = 0; c < NC; c++) e.w[c] = fw[c];
            e.m = fm;
        };
        // Z rows of every antenna for one stage (as in k_herk_fused's producers)
        auto produce = [&](unsigned char *buf, int stage) {
            const SrcEntry<NC> &se = src[stage & 1][msl];
            const int64_t m = se.m;
            const bool lv = m >= 0;
            const double x0 = se.x, x1 = se.y, x2 = se.z;
            float2 wl[NC];
            for (int c = 0; c < NC; c++) wl[c] = se.w[c];
            const bool multi_beam = a.n_beam != 1;
            int cur_b = multi_beam ? -1 : 0;
            // not unrolled: the accumulators stay live across this loop
#pragma unroll 1
            for (int as = g; as < NA; as += NG) {
                const AntEntry e = tab[as];
                if (multi_beam && lv && e.b >= 0 && e.b != cur_b) {
                    for (int c = 0; c < NC; c++) wl[c] = Bm[((int64_t)e.b * NC + c) * a.ld_src + m];
                    cur_b = e.b;
                }
                const double p = e.ux * x0 + e.uy * x1 + e.uz * x2;
                const float r = (float)(p - rint(p));
                const float msk = (lv && e.b >= 0) ? 1.0f : 0.0f;
                const float sn = msk * __builtin_amdgcn_sinf(-r);
                const float cs = msk * __builtin_amdgcn_cosf(-r);
                float2 z[NC];
                for (int c = 0; c < NC; c++) {
                    z[c].x = wl[c].x * cs - wl[c].y * sn;
                    z[c].y = wl[c].x * sn + wl[c].y * cs;
                }
#pragma unroll
                for (int p = 0; p < NF; p++) {
                    unsigned char *row = buf + (as * NF + p) * RS;
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
                }
            }
        };

        f32x4 acc_re[18], acc_im[18];
        for (int t = 0; t < 18; t++)
            for (int e = 0; e < 4; e++) {
                acc_re[t][e] = 0.f;
                acc_im[t][e] = 0.f;
            }
        auto consume = [&](const unsigned char *buf) {
            if (sq)
                consume_sq_b3<GeomPair>(buf, sq_rb, sq_cb, l16, lk, acc_re, acc_im);
            else if (tri_s == 0)
                consume_tri_b3<GeomPair, TriSet<0>>(buf, tri_o, l16, lk, acc_re, acc_im);
            else
                consume_tri_b3<GeomPair, TriSet<1>>(buf, tri_o, l16, lk, acc_re, acc_im);
        };

        if (fetcher) {
            fetch(0);
            stash(0);
            fetch(1);
            stash(1);
        }
        __syncthreads();  // antenna table and the first two stages' sources ready
        produce(lds, 0);
        __syncthreads();
        for (int stg = 0; stg < n_stage; stg++) {
            unsigned char *cur = lds + (stg & 1) * L::BUF;
            unsigned char *nxt = lds + ((stg + 1) & 1) * L::BUF;
            const bool more = stg + 1 < n_stage;
            if (fetcher && stg + 2 < n_stage) fetch(stg + 2);
            if (sq) consume(cur);
            if (more) produce(nxt, stg + 1);
            if (!sq) consume(cur);
            // src[stg & 1] was last read by the producers of stage stg (one stage ago)
            if (fetcher && stg + 2 < n_stage) stash(stg + 2);
            __syncthreads();
        }

        // the write-out offsets are recomputed here rather than kept live across the item
        int ld = Np;
        asm volatile("" : "+v"(ld));
        float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
        if (sq) {
            const int r0 = 16 * sq_rb + 4 * lk, c0 = 16 * sq_cb + l16;
#pragma unroll
            for (int i = 0; i < kTI; i++)
#pragma unroll
                for (int j = 0; j < kTI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        P[(int64_t)(r0 + 16 * i + e) * ld + c0 + 16 * j] =
                            make_float2(acc_re[i * kTI + j][e], acc_im[i * kTI + j][e]);
        } else {
            // slot t: row k of the set with base[k] <= t < base[k] + r[k] + 1, column t - base[k]
            const int rows[4] = {tri_s == 0 ? 0 : 2, tri_s == 0 ? 7 : 5, tri_s == 0 ? 1 : 3, tri_s == 0 ? 6 : 4};
#pragma unroll
            for (int t = 0; t < 18; t++) {
                int k = 0, b = 0;
                while (t >= b + rows[k] + 1) {
                    b += rows[k] + 1;
                    k++;
                }
                const int R = rows[k], C = t - b;
                const int r0 = tri_o + 16 * R + 4 * lk, c0 = tri_o + 16 * C + l16;
#pragma unroll
                for (int e = 0; e < 4; e++) P[(int64_t)(r0 + e) * ld + c0] = make_float2(acc_re[t][e], acc_im[t][e]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Polarised products with one shared beam (BF16X3 or FP32, 2 feeds x 2 axes,
// more than 64 antennas).  With Z[(a,p),(m,k)] = B_pk(m) F_a(m) (F the fringe factor of
// antenna a, B = sqrt(I) A the same for every antenna), the sum over the
// axis index k can be taken per source first:
//   V[(a,p),(b,q)] = sum_m F_a(m) conj(F_b(m)) C_pq(m),
//   C_pq(m) = sum_k B_pk(m) conj(B_qk(m))   (the 2 x 2 coherency seen through the beam).
// With s0 = sqrt(C_00), s1 = sqrt(C_11), l = C_10 / s0 (|l| <= s1 by
// Cauchy-Schwarz; l = 0 where s0 = 0, where C_10 = 0 too) and three operand
// planes over the antennas
//   P0 = s0 F,  P1 = s1 F,  L = l F,
// the three independent feed blocks are V^00 = P0 P0^H, V^11 = P1 P1^H (lower
// triangles) and V^10 = L P0^H (full), and V^01 = (V^10)^H.  The product runs
// over the sources instead of the (source, axis) columns of Z: half the
// multiply-adds of Z Z^H for the same result.
//
// Layout: up to 512 staged rows per stage (plane * 128 + antenna), 16 sources
// per stage.  Antennas come in blocks of 128.  A diagonal item (block I)
// stages P0, P1, L of the block; its waves and tiles are those of
// k_herk_b3_pair: the square waves take V^10 (rows of L against rows of P0),
// the triangle waves V^00 and V^11.  An off-diagonal item (blocks I > J, a
// launch of its own) stages two planes of both blocks and computes two full
// 128 x 128 products, a 64 x 64 quadrant per wave: kind X, P0_I P0_J^H and
// P1_I P1_J^H; kind Y, L_I P0_J^H and L_J P0_I^H.  V^10 elements with a < b
// are stored, conjugated, at the transposed lower position of the
// (a, p) x (b, q) matrix, which is where the reduction reads them.
// ---------------------------------------------------------------------------
struct CohSrc {
    double x, y, z;  // s_hat
    float s0, s1;    // sqrt C00, sqrt C11
    float lx, ly;    // C10 / sqrt C00 (all four 0 past the split)
};

template <int PREC, bool OFF, int SQ_ANT = 96, bool SHORT = false>
__global__ void __launch_bounds__(512, 1) k_herk_coh(FusedArgs a) {
    // 144-byte rows: hi + lo bf16 planes, or one complex64 plane (FP32); 160 bytes
    // on the three-plane diagonal items of BF16X3
    constexpr bool R160 = !OFF && PREC == PB3;
    typedef typename std::conditional<R160, GeomCoh3, GeomCoh>::type L;
    constexpr int RS = L::RS;
    constexpr int SPS = 16;                 // sources per stage
    constexpr int ROWS = (OFF ? 4 : 3) * kST;  // planes of 128 antennas
    constexpr int BUF = ROWS * RS;
    // SQ_ANT: antennas formed by the square waves (the rest by the triangle waves,
    // which have more products per stage); the split evens out the two waves of a
    // SIMD, 96 by default, 64 as a tuning variant.
    static_assert(SQ_ANT % 32 == 0 && (kST - SQ_ANT) % 32 == 0, "32 antennas per pass of a wave group");
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];
    __shared__ AntEntry tab[2 * kST];
    __shared__ CohSrc src[2][SPS];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const bool sq = wave < 4;
    const int l16 = lane & 15, lk = lane >> 4;
    const int Np = a.n_rows_pad;
    // Antenna blocks of 128: per (instance, k-split), one item per diagonal block
    // I (V^00_II, V^11_II triangles and V^10_II; OFF = false) and two per block
    // pair I > J (OFF = true, a launch of its own): kind X, V^00_IJ = P0_I P0_J^H
    // and V^11_IJ = P1_I P1_J^H; kind Y, V^10_IJ = L_I P0_J^H and V^10_JI =
    // L_J P0_I^H (the conjugate of the (0, 1) entries).
    const int nb = Np / (2 * kST);
    // A last diagonal block of at most 96 antennas (a short block) has a launch of
    // its own (SHORT): six tile rows, the square waves 3 x 3 tiles of V^10 each and
    // the triangle waves the row sets of TriSet6; its square waves form 64
    // antennas and its triangle waves 32.  The other launch skips that block.
    constexpr bool short_blk = SHORT;
    const bool has_short = !OFF && a.n_ant - (nb - 1) * kST <= 96;
    const int n_kind = OFF ? nb * (nb - 1) : SHORT ? 1 : has_short ? nb - 1 : nb;
    const int total = a.work[a.n_inst] * n_kind;
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int mp = tid % (SPS / 2);  // source pair
    const int a0o = wrow(tid);  // off-diagonal items: antennas a0o + 64 k of the 256 of blocks I, J
    // this thread's antennas: a0, a0 + 32, ... (SQ_ANT / 32 of them, or (kST - SQ_ANT) / 32)
    const int a0 = sq ? (R160 ? wrow160(tid) : wrow(tid)) : SQ_ANT + (R160 ? wrow160(tid - 256) : wrow(tid - 256));
    // square waves: V^10 rows 16 (sq_rb + i) of L against 16 (sq_cb + j) of P0 (block units)
    const int sq_r0 = 4 * (wave >> 1), sq_c0 = 4 * (wave & 1);
    const int sq_rb = 2 * 8 + sq_r0, sq_cb = sq_c0;
    const int sh_r0 = 3 * (wave >> 1), sh_c0 = 3 * (wave & 1);  // short diagonal block: 3 x 3 tiles
    // triangle waves: plane T (V^TT), row set S
    const int tri_t = (wave - 4) >> 1, tri_s = (wave - 4) & 1;
    const int tri_o = tri_t * kST;

    for (int item = slot_x; item < total; item += a.grid) {
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work[mid] * n_kind <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int inst = lo;
        const int local = item - a.work[inst] * n_kind;
        const int s = local / n_kind;
        const int kind = local % n_kind;
        constexpr bool off = OFF;
        const bool kind_y = off && (kind & 1);
        int I = SHORT ? nb - 1 : kind, J = I;
        if (off) {  // pairs (1, 0), (2, 0), (2, 1), (3, 0), ...
            int q = kind >> 1;
            I = 1;
            while (q >= I) {
                q -= I;
                I++;
            }
            J = q;
        }
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.kcols[inst] / 2;
        const int64_t m_begin = (int64_t)s * ms_per_split;
        const int64_t m_end = m_begin + ms_per_split < M ? m_begin + ms_per_split : M;
        const int n_stage = (int)((m_end - m_begin + SPS - 1) / SPS);
        const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
        const float2 *Bm = (const float2 *)a.B + (int64_t)inst * 4 * a.ld_src;

        {
            const double nu_c = a.freqs[f] / kSpeedOfLight;
            for (int as = tid; as < (off ? 2 : 1) * kST; as += 512) {
                const int ant = as < kST ? I * kST + as : J * kST + (as - kST);
                AntEntry e;
                if (ant < a.n_ant) {
                    e.ux = nu_c * a.antc[3 * ant];
                    e.uy = nu_c * a.antc[3 * ant + 1];
                    e.uz = nu_c * a.antc[3 * ant + 2];
                    e.b = 0;
                } else {
                    e.ux = e.uy = e.uz = 0.0;
                    e.b = -1;
                }
                e.pad = 0;
                tab[as] = e;
            }
        }

        // per-source direction and coherency factors, loaded and formed one stage
        // ahead by the first SPS lanes of wave 0
        const bool fetcher = tid < SPS;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        float2 fb[4];
        int fm = -1;
        auto fetch = [&](int stage) {
            const int64_t m = m_begin + (int64_t)stage * SPS + tid;
            fm = (stage < n_stage && m < m_end) ? (int)m : -1;
            fx = fy = fz = 0.0;
            for (int c = 0; c < 4; c++) fb[c] = make_float2(0.f, 0.f);
            if (fm >= 0) {
                fx = sh[fm];
                fy = sh[a.ld_src + fm];
                fz = sh[2 * a.ld_src + fm];
                for (int c = 0; c < 4; c++) fb[c] = Bm[(int64_t)c * a.ld_src + fm];
            }
        };
        auto stash = [&](int stage) {
            // B components c = 2 p + k
            const float c00 = fb[0].x * fb[0].x + fb[0].y * fb[0].y + fb[1].x * fb[1].x + fb[1].y * fb[1].y;
            const float c11 = fb[2].x * fb[2].x + fb[2].y * fb[2].y + fb[3].x * fb[3].x + fb[3].y * fb[3].y;
            // C10 = B10 conj(B00) + B11 conj(B01)
            const float c10x = fb[2].x * fb[0].x + fb[2].y * fb[0].y + fb[3].x * fb[1].x + fb[3].y * fb[1].y;
            const float c10y = fb[2].y * fb[0].x - fb[2].x * fb[0].y + fb[3].y * fb[1].x - fb[3].x * fb[1].y;
            const float s0 = sqrtf(c00);
            CohSrc &e = src[stage & 1][tid];
            e.x = fx;
            e.y = fy;
            e.z = fz;
            e.s0 = s0;
            e.s1 = sqrtf(c11);
            e.lx = s0 > 0.f ? c10x / s0 : 0.f;
            e.ly = s0 > 0.f ? c10y / s0 : 0.f;
        };
        // The three planes of this thread's two sources for its NA antennas.  No
        // masks: a source past the split has zero coherency factors, and rows of
        // padding antennas (u = 0) only reach outputs that are never stored.
        auto produce_n = [&](unsigned char *buf, int stage, auto na, int a0) {
            constexpr int NA = decltype(na)::value;
            CohSrc w[2];
            w[0] = src[stage & 1][2 * mp];
            w[1] = src[stage & 1][2 * mp + 1];
            AntEntry ee[NA];
#pragma unroll
            for (int k = 0; k < NA; k++) ee[k] = tab[a0 + 32 * k];
#pragma unroll
            for (int k = 0; k < NA; k++) {
                const int as = a0 + 32 * k;
                const AntEntry &e = ee[k];
                uint32_t h[3][2], l[3][2];
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const double p = e.ux * w[q].x + e.uy * w[q].y + e.uz * w[q].z;
                    const float r = (float)__builtin_amdgcn_fract(p);
                    const float fi = __builtin_amdgcn_sinf(-r);
                    const float fr = __builtin_amdgcn_cosf(-r);
                    if constexpr (PREC == PB3) {
                        split2(w[q].s0 * fr, w[q].s0 * fi, h[0][q], l[0][q]);
                        split2(w[q].s1 * fr, w[q].s1 * fi, h[1][q], l[1][q]);
                        split2(w[q].lx * fr - w[q].ly * fi, w[q].lx * fi + w[q].ly * fr, h[2][q], l[2][q]);
                    } else {  // FP32: (re, im) words of each plane
                        h[0][q] = __float_as_uint(w[q].s0 * fr);
                        l[0][q] = __float_as_uint(w[q].s0 * fi);
                        h[1][q] = __float_as_uint(w[q].s1 * fr);
                        l[1][q] = __float_as_uint(w[q].s1 * fi);
                        h[2][q] = __float_as_uint(w[q].lx * fr - w[q].ly * fi);
                        l[2][q] = __float_as_uint(w[q].lx * fi + w[q].ly * fr);
                    }
                }
#pragma unroll
                for (int pl = 0; pl < 3; pl++) {
                    if constexpr (PREC == PB3) {
                        unsigned char *row = buf + (pl * kST + as) * RS + mp * 8;
                        *(uint2 *)row = make_uint2(h[pl][0], h[pl][1]);
                        *(uint2 *)(row + L::PLANEB) = make_uint2(l[pl][0], l[pl][1]);
                    } else {  // two complex64 of sources 2 mp, 2 mp + 1
                        unsigned char *row = buf + (pl * kST + as) * RS + mp * 16;
                        *(u32x4 *)row = u32x4{h[pl][0], l[pl][0], h[pl][1], l[pl][1]};
                    }
                }
            }
        };
        // Off-diagonal items: two planes of each of the 256 antennas of blocks I, J
        // (X: P0, P1; Y: L, P0), block I in planes 0-1, block J in planes 2-3.
        auto produce_off = [&](unsigned char *buf, int stage) {
            CohSrc w[2];
            w[0] = src[stage & 1][2 * mp];
            w[1] = src[stage & 1][2 * mp + 1];
            AntEntry ee[4];
#pragma unroll
            for (int k = 0; k < 4; k++) ee[k] = tab[a0o + 64 * k];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int as = a0o + 64 * k;
                const int pl0 = 2 * (as >> 7), row = as & (kST - 1);
                float vr[2][2], vi[2][2];
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const double p = ee[k].ux * w[q].x + ee[k].uy * w[q].y + ee[k].uz * w[q].z;
                    const float r = (float)__builtin_amdgcn_fract(p);
                    const float fi = __builtin_amdgcn_sinf(-r);
                    const float fr = __builtin_amdgcn_cosf(-r);
                    if (kind_y) {
                        vr[0][q] = w[q].lx * fr - w[q].ly * fi;
                        vi[0][q] = w[q].lx * fi + w[q].ly * fr;
                        vr[1][q] = w[q].s0 * fr;
                        vi[1][q] = w[q].s0 * fi;
                    } else {
                        vr[0][q] = w[q].s0 * fr;
                        vi[0][q] = w[q].s0 * fi;
                        vr[1][q] = w[q].s1 * fr;
                        vi[1][q] = w[q].s1 * fi;
                    }
                }
#pragma unroll
                for (int v = 0; v < 2; v++) {
                    if constexpr (PREC == PB3) {
                        uint32_t h0, l0, h1, l1;
                        split2(vr[v][0], vi[v][0], h0, l0);
                        split2(vr[v][1], vi[v][1], h1, l1);
                        unsigned char *rp = buf + ((pl0 + v) * kST + row) * RS + mp * 8;
                        *(uint2 *)rp = make_uint2(h0, h1);
                        *(uint2 *)(rp + L::PLANEB) = make_uint2(l0, l1);
                    } else {
                        unsigned char *rp = buf + ((pl0 + v) * kST + row) * RS + mp * 16;
                        *(u32x4 *)rp = u32x4{__float_as_uint(vr[v][0]), __float_as_uint(vi[v][0]),
                                             __float_as_uint(vr[v][1]), __float_as_uint(vi[v][1])};
                    }
                }
            }
        };
        auto produce = [&](unsigned char *buf, int stage) {
            if constexpr (OFF)
                produce_off(buf, stage);
            else if (short_blk && sq)
                produce_n(buf, stage, std::integral_constant<int, 2>{}, R160 ? wrow160(tid) : wrow(tid));
            else if (short_blk)
                produce_n(buf, stage, std::integral_constant<int, 1>{}, 64 + (R160 ? wrow160(tid - 256) : wrow(tid - 256)));
            else if (sq)
                produce_n(buf, stage, std::integral_constant<int, SQ_ANT / 32>{}, a0);
            else
                produce_n(buf, stage, std::integral_constant<int, (kST - SQ_ANT) / 32>{}, a0);
        };

        constexpr int NACC = OFF ? 16 : 18;
        f32x4 acc_re[NACC], acc_im[NACC];
        for (int t = 0; t < NACC; t++)
            for (int e = 0; e < 4; e++) {
                acc_re[t][e] = 0.f;
                acc_im[t][e] = 0.f;
            }
        // off-diagonal items: wave w takes quadrant w & 3 of product w >> 2
        const int o_rp = !kind_y ? (wave >> 2) : (wave < 4 ? 0 : 2);       // row plane
        const int o_cp = !kind_y ? 2 + (wave >> 2) : (wave < 4 ? 3 : 1);  // column plane
        const int o_rb = o_rp * 8 + 4 * ((wave & 3) >> 1), o_cb = o_cp * 8 + 4 * (wave & 1);
        auto consume = [&](const unsigned char *buf) {
            if constexpr (OFF) {
                if constexpr (PREC == PB3)
                    consume_sq_b3<L>(buf, o_rb, o_cb, l16, lk, acc_re, acc_im);
                else
                    consume_sq_f32<L>(buf, o_rb, o_cb, l16, lk, acc_re, acc_im);
            } else if constexpr (PREC == PB3) {
                if (short_blk && sq)
                    consume_sq_b3<L, NACC, 3, 3>(buf, 16 + sh_r0, sh_c0, l16, lk, acc_re, acc_im);
                else if (short_blk && tri_s == 0)
                    consume_tri_b3<L, TriSet6<0>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else if (short_blk)
                    consume_tri_b3<L, TriSet6<1>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else if (sq)
                    consume_sq_b3<L>(buf, sq_rb, sq_cb, l16, lk, acc_re, acc_im);
                else if (tri_s == 0)
                    consume_tri_b3<L, TriSet<0>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else
                    consume_tri_b3<L, TriSet<1>>(buf, tri_o, l16, lk, acc_re, acc_im);
            } else {
                if (short_blk && sq)
                    consume_sq_f32<L, NACC, 3, 3>(buf, 16 + sh_r0, sh_c0, l16, lk, acc_re, acc_im);
                else if (short_blk && tri_s == 0)
                    consume_tri_f32<L, TriSet6<0>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else if (short_blk)
                    consume_tri_f32<L, TriSet6<1>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else if (sq)
                    consume_sq_f32<L>(buf, sq_rb, sq_cb, l16, lk, acc_re, acc_im);
                else if (tri_s == 0)
                    consume_tri_f32<L, TriSet<0>>(buf, tri_o, l16, lk, acc_re, acc_im);
                else
                    consume_tri_f32<L, TriSet<1>>(buf, tri_o, l16, lk, acc_re, acc_im);
            }
        };

        if (fetcher) {
            fetch(0);
            stash(0);
            fetch(1);
            stash(1);
        }
        __syncthreads();  // antenna table and the first two stages' sources ready
        produce(lds, 0);
        __syncthreads();
        for (int stg = 0; stg < n_stage; stg++) {
            unsigned char *cur = lds + (stg & 1) * BUF;
            unsigned char *nxt = lds + ((stg + 1) & 1) * BUF;
            const bool more = stg + 1 < n_stage;
            if (fetcher && stg + 2 < n_stage) fetch(stg + 2);
            if (sq) consume(cur);
            if (more) produce(nxt, stg + 1);
            if (!sq) consume(cur);
            // src[stg & 1] was last read by the producers of stage stg (one stage ago)
            if (fetcher && stg + 2 < n_stage) stash(stg + 2);
            __syncthreads();
        }

        int ld = Np;
        asm volatile("" : "+v"(ld));
        float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
        if constexpr (OFF) {
            // rows of the product: antennas of block (Y, waves 4-7: J, else I); columns: the other block
            const int rblk = kind_y && wave >= 4 ? J : I, cblk = kind_y && wave >= 4 ? I : J;
            const int r0 = 4 * ((wave & 3) >> 1), c0 = 4 * (wave & 1);
#pragma unroll
            for (int i = 0; i < kTI; i++)
#pragma unroll
                for (int j = 0; j < kTI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int A = rblk * kST + 16 * (r0 + i) + 4 * lk + e, Bc = cblk * kST + 16 * (c0 + j) + l16;
                        const float vr = acc_re[i * kTI + j][e], vi = acc_im[i * kTI + j][e];
                        if (A >= a.n_ant || Bc >= a.n_ant) continue;
                        if (!kind_y)  // V^pp, p = wave >> 2: rows 2 A + p > columns 2 Bc + p
                            P[(int64_t)(2 * A + (wave >> 2)) * ld + 2 * Bc + (wave >> 2)] = make_float2(vr, vi);
                        else if (wave < 4)  // V^10 with A in I > Bc in J
                            P[(int64_t)(2 * A + 1) * ld + 2 * Bc] = make_float2(vr, vi);
                        else  // V^10 with A in J < Bc in I: the conjugate at (2 Bc, 2 A + 1)
                            P[(int64_t)(2 * Bc) * ld + 2 * A + 1] = make_float2(vr, -vi);
                    }
        } else if (sq) {
            // V^10 tile (R, C) of the block from slot i * kTI + j
            const int nt = short_blk ? 3 : kTI, r0 = short_blk ? sh_r0 : sq_r0, c0 = short_blk ? sh_c0 : sq_c0;
#pragma unroll
            for (int i = 0; i < kTI; i++)
#pragma unroll
                for (int j = 0; j < kTI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int ra = I * kST + 16 * (r0 + i) + 4 * lk + e, cb = I * kST + 16 * (c0 + j) + l16;
                        const float vr = acc_re[i * kTI + j][e], vi = acc_im[i * kTI + j][e];
                        if (i >= nt || j >= nt || ra >= a.n_ant || cb >= a.n_ant) continue;
                        if (ra >= cb)
                            P[(int64_t)(2 * ra + 1) * ld + 2 * cb] = make_float2(vr, vi);
                        else
                            P[(int64_t)(2 * cb) * ld + 2 * ra + 1] = make_float2(vr, -vi);
                    }
        } else {
            // V^TT tile (R, C) of the block, R >= C, from its triangle slot
            auto store = [&](int t, int R, int C) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int ra = I * kST + 16 * R + 4 * lk + e, cb = I * kST + 16 * C + l16;
                    if (ra >= a.n_ant || cb >= a.n_ant) continue;
                    P[(int64_t)(2 * ra + tri_t) * ld + 2 * cb + tri_t] = make_float2(acc_re[t][e], acc_im[t][e]);
                }
            };
            if (short_blk) {
                if (tri_s == 0)
                    for_tri_tiles<TriSet6<0>>(store);
                else
                    for_tri_tiles<TriSet6<1>>(store);
            } else {
                if (tri_s == 0)
                    for_tri_tiles<TriSet<0>>(store);
                else
                    for_tri_tiles<TriSet<1>>(store);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Off-diagonal block pairs of the product over sources (BF16X3) with the
// per-source weight on one side.  For antenna blocks I > J each of the four
// block products is
//   sum_m w(m) F_a(m) conj(F_b(m)) = ((w F_I) F_J^H)[a, b],  a in I, b in J,
// with w = C_00, C_11 (kind X: V^00_IJ, V^11_IJ), or w = C_10 and conj C_10
// (kind Y: V^10_IJ, and V^01_IJ = the Hermitian partner of V^10_JI).  So the
// columns of both products of an item are the unweighted fringe rows F_J, formed
// and split once, and only the rows carry the weights.  A stage holds four
// planes of 128 rows x 16 sources: w0 F_I, w1 F_I, F_J, and F_J rotated,
// (re, im) -> (-im, re), for the imaginary parts, written at forming time so the
// multiply loop runs its MFMAs on LDS operands with no vector work on them.
// Rows are 160 bytes (conflict-free 16-byte operand reads), so two stages fill
// the 160 KB of LDS; the antenna table and the per-source weights live in the
// 32 unused bytes at the end of rows, which the forming never writes and the
// multiply never reads.  Against k_herk_coh<PREC, true> (both operands weighted
// by square roots of the coherency) that is a quarter fewer rows to scale and
// split per stage.
//
// Waves s and s + 4 share SIMD s: wave s takes product 0 and row half s >> 1 of
// the 128 x 128 block, wave s + 4 product 1 and the other row half, both column
// half s & 1 (16 tiles of 16 x 16 each).  When block I is the last, short block,
// tile rows past its antennas are neither formed nor multiplied, and its row
// tiles are split evenly between the halves (3 + 3 for 94 antennas), so the two
// waves of a SIMD still carry equal products and their multiply and forming
// phases keep overlapping; an uneven split (4 + 2) leaves the lighter wave
// idle at every barrier.
// ---------------------------------------------------------------------------
// Per-source direction and the item's two weights: (C_00, C_11) for kind X,
// (Re, Im) of C_10 for kind Y, with C_pq = sum_k B_pk conj(B_qk) (0 past the split)
struct PairSrc {
    double x, y, z;  // s_hat
    float w0, w1;
};

// Rows 16 (rb + i), i < NR, of one plane against columns 16 (cb + j) and their
// rotations 16 (wb + j), j < 4: re += a b, im += a rot(b) for the hi / lo terms.
template <typename L, int NR>
__device__ __forceinline__ void consume_pairs_b3(const unsigned char *buf, int rb, int cb, int wb, int l16, int lk,
                                                 f32x4 (&re)[16], f32x4 (&im)[16]) {
    // loads in the order of first use: hi rows, the first column's hi terms, lo
    // terms, lo rows
    u32x4 ah[NR], al[NR];
#pragma unroll
    for (int i = 0; i < NR; i++) ah[i] = *(const u32x4 *)(buf + (16 * (rb + i) + l16) * L::RS + lk * 16);
    const unsigned char *pc = buf + (16 * cb + l16) * L::RS + lk * 16;
    const unsigned char *pw = buf + (16 * wb + l16) * L::RS + lk * 16;
    u32x4 nh = *(const u32x4 *)pc, mh = *(const u32x4 *)pw;
    u32x4 nl = *(const u32x4 *)(pc + L::PLANEB), ml = *(const u32x4 *)(pw + L::PLANEB);
#pragma unroll
    for (int i = 0; i < NR; i++) al[i] = *(const u32x4 *)(buf + (16 * (rb + i) + l16) * L::RS + lk * 16 + L::PLANEB);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kTI; j++) {
        const u32x4 bh = nh, bl = nl, wh = mh, wl = ml;
        if (j + 1 < kTI) {
            const unsigned char *q = pc + 16 * (j + 1) * L::RS, *r = pw + 16 * (j + 1) * L::RS;
            nh = *(const u32x4 *)q;
            mh = *(const u32x4 *)r;
            nl = *(const u32x4 *)(q + L::PLANEB);
            ml = *(const u32x4 *)(r + L::PLANEB);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NR; i++) mfma_pair(ah[i], bh, wh, re[i * kTI + j], im[i * kTI + j]);
#pragma unroll
        for (int i = 0; i < NR; i++) mfma_pair(ah[i], bl, wl, re[i * kTI + j], im[i * kTI + j]);
#pragma unroll
        for (int i = 0; i < NR; i++) mfma_pair(al[i], bh, wh, re[i * kTI + j], im[i * kTI + j]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__global__ void __launch_bounds__(512, 1) k_herk_pairs(FusedArgs a) {
    typedef GeomCoh3 L;
    constexpr int RS = L::RS;
    constexpr int SPS = 16;         // sources per stage
    constexpr int BUF = 4 * kST * RS;
    constexpr int PAD = 2 * L::PLANEB;  // the unused end of a row
    static_assert(2 * BUF <= 160 * 1024, "two stages exceed the LDS");
    static_assert(sizeof(AntEntry) <= RS - PAD && sizeof(PairSrc) <= RS - PAD, "row padding too small");
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];
    // antenna entry as (of the 256 of blocks I, J) at the end of row as of stage 0;
    // the sources of stage parity st at the end of rows 16 st + m of stage 1
    auto tab = [&](int as) -> AntEntry & { return *(AntEntry *)(lds + as * RS + PAD); };
    auto src = [&](int st, int m) -> PairSrc & { return *(PairSrc *)(lds + BUF + (SPS * st + m) * RS + PAD); };

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const int l16 = lane & 15, lk = lane >> 4;
    const int Np = a.n_rows_pad;
    const int nb = Np / (2 * kST);
    const int n_kind = nb * (nb - 1);  // two kinds per block pair
    const int total = a.work[a.n_inst] * n_kind;
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int mp = tid % (SPS / 2);   // source pair 2 mp, 2 mp + 1
    const int simd = wave & 3, pr = wave >> 2;
    const int rh = (simd >> 1) ^ pr, ch = simd & 1;
    const int a0 = wrow160(tid);      // antennas a0 + 64 k of the 256 of blocks I (k < 2) and J
    const int o_cb = 2 * 8 + 4 * ch, o_wb = 3 * 8 + 4 * ch;
    const bool mult_first = wave < 4;

    for (int item = slot_x; item < total; item += a.grid) {
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work[mid] * n_kind <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int inst = lo;
        const int local = item - a.work[inst] * n_kind;
        const int s = local / n_kind;
        const int kind = local % n_kind;
        const bool kind_y = kind & 1;
        int q = kind >> 1, I = 1;  // pairs (1, 0), (2, 0), (2, 1), (3, 0), ...
        while (q >= I) {
            q -= I;
            I++;
        }
        const int J = q;
        const int n_i = a.n_ant - I * kST < kST ? a.n_ant - I * kST : kST;  // antennas of block I
        // row tiles of block I (8, or fewer on the short last block), split evenly
        // between the row halves so the two waves of a SIMD multiply alike
        const int nt = (n_i + 15) / 16, nt0 = (nt + 1) / 2;
        const int r0 = rh ? nt0 : 0, nrt = rh ? nt - nt0 : nt0;  // this wave's first tile and count
        const int o_rb = pr * 8 + r0;
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.kcols[inst] / 2;
        const int64_t m_begin = (int64_t)s * ms_per_split;
        const int64_t m_end = m_begin + ms_per_split < M ? m_begin + ms_per_split : M;
        const int n_stage = (int)((m_end - m_begin + SPS - 1) / SPS);
        const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
        const float2 *Bm = (const float2 *)a.B + (int64_t)inst * 4 * a.ld_src;

        {
            const double nu_c = a.freqs[f] / kSpeedOfLight;
            for (int as = tid; as < 2 * kST; as += 512) {
                const int ant = as < kST ? I * kST + as : J * kST + (as - kST);
                AntEntry e;
                if (ant < a.n_ant) {
                    e.ux = nu_c * a.antc[3 * ant];
                    e.uy = nu_c * a.antc[3 * ant + 1];
                    e.uz = nu_c * a.antc[3 * ant + 2];
                    e.b = 0;
                } else {
                    e.ux = e.uy = e.uz = 0.0;
                    e.b = -1;
                }
                e.pad = 0;
                tab(as) = e;
            }
        }

        // per-source direction and coherency, loaded and formed one stage ahead by
        // the first SPS lanes of wave 0
        const bool fetcher = tid < SPS;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        float2 fb[4];
        auto fetch = [&](int stage) {
            const int64_t m = m_begin + (int64_t)stage * SPS + tid;
            const bool ok = stage < n_stage && m < m_end;
            fx = fy = fz = 0.0;
            for (int c = 0; c < 4; c++) fb[c] = make_float2(0.f, 0.f);
            if (ok) {
                fx = sh[m];
                fy = sh[a.ld_src + m];
                fz = sh[2 * a.ld_src + m];
                for (int c = 0; c < 4; c++) fb[c] = Bm[(int64_t)c * a.ld_src + m];
            }
        };
        auto stash = [&](int stage, bool ky) {
            PairSrc &e = src(stage & 1, tid);
            e.x = fx;
            e.y = fy;
            e.z = fz;
            // B components c = 2 p + k; C_10 = B_10 conj(B_00) + B_11 conj(B_01)
            if (ky) {
                e.w0 = fb[2].x * fb[0].x + fb[2].y * fb[0].y + fb[3].x * fb[1].x + fb[3].y * fb[1].y;
                e.w1 = fb[2].y * fb[0].x - fb[2].x * fb[0].y + fb[3].y * fb[1].x - fb[3].x * fb[1].y;
            } else {
                e.w0 = fb[0].x * fb[0].x + fb[0].y * fb[0].y + fb[1].x * fb[1].x + fb[1].y * fb[1].y;
                e.w1 = fb[2].x * fb[2].x + fb[2].y * fb[2].y + fb[3].x * fb[3].x + fb[3].y * fb[3].y;
            }
        };
        // Weighted rows of block I (planes 0, 1) or plain and rotated rows of block
        // J (planes 2, 3) for this thread's two sources.  Rows of block I past its
        // antennas are skipped (never multiplied); a source past the split has zero
        // weights, and its J rows only meet zero-weighted I rows.
        auto produce = [&](unsigned char *buf, int stage, auto ky) {
            constexpr bool KY = decltype(ky)::value;
            PairSrc w[2];
            w[0] = src(stage & 1, 2 * mp);
            w[1] = src(stage & 1, 2 * mp + 1);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int as = a0 + 64 * k;
                const bool in_i = k < 2;
                if (in_i && as >= n_i) continue;
                const AntEntry e = tab(as);
                float fr[2], fi[2];
#pragma unroll
                for (int qq = 0; qq < 2; qq++) {
                    const double p = e.ux * w[qq].x + e.uy * w[qq].y + e.uz * w[qq].z;
                    const float r = (float)__builtin_amdgcn_fract(p);
                    fi[qq] = __builtin_amdgcn_sinf(-r);
                    fr[qq] = __builtin_amdgcn_cosf(-r);
                }
                if (in_i) {
                    uint32_t h0[2], l0[2], h1[2], l1[2];
#pragma unroll
                    for (int qq = 0; qq < 2; qq++) {
                        if constexpr (KY) {  // w0 = C_10, w1 = conj C_10
                            const float cx = w[qq].w0, cy = w[qq].w1;
                            split2(cx * fr[qq] - cy * fi[qq], cx * fi[qq] + cy * fr[qq], h0[qq], l0[qq]);
                            split2(cx * fr[qq] + cy * fi[qq], cx * fi[qq] - cy * fr[qq], h1[qq], l1[qq]);
                        } else {  // w0 = C_00, w1 = C_11
                            split2(w[qq].w0 * fr[qq], w[qq].w0 * fi[qq], h0[qq], l0[qq]);
                            split2(w[qq].w1 * fr[qq], w[qq].w1 * fi[qq], h1[qq], l1[qq]);
                        }
                    }
                    unsigned char *r0 = buf + as * RS + mp * 8, *r1 = buf + (kST + as) * RS + mp * 8;
                    *(uint2 *)r0 = make_uint2(h0[0], h0[1]);
                    *(uint2 *)(r0 + L::PLANEB) = make_uint2(l0[0], l0[1]);
                    *(uint2 *)r1 = make_uint2(h1[0], h1[1]);
                    *(uint2 *)(r1 + L::PLANEB) = make_uint2(l1[0], l1[1]);
                } else {
                    uint32_t h[2], l[2];
#pragma unroll
                    for (int qq = 0; qq < 2; qq++) split2(fr[qq], fi[qq], h[qq], l[qq]);
                    const int rj = as - kST;  // row of block J
                    unsigned char *r2 = buf + (2 * kST + rj) * RS + mp * 8, *r3 = buf + (3 * kST + rj) * RS + mp * 8;
                    *(uint2 *)r2 = make_uint2(h[0], h[1]);
                    *(uint2 *)(r2 + L::PLANEB) = make_uint2(l[0], l[1]);
                    // (re, im) -> (-im, re) on each bf16 pair: swap the halves, negate the low one
                    *(uint2 *)r3 = make_uint2(__builtin_amdgcn_alignbit(h[0], h[0], 16) ^ 0x00008000u,
                                              __builtin_amdgcn_alignbit(h[1], h[1], 16) ^ 0x00008000u);
                    *(uint2 *)(r3 + L::PLANEB) = make_uint2(__builtin_amdgcn_alignbit(l[0], l[0], 16) ^ 0x00008000u,
                                                            __builtin_amdgcn_alignbit(l[1], l[1], 16) ^ 0x00008000u);
                }
            }
        };

        f32x4 acc_re[16], acc_im[16];
        for (int t = 0; t < 16; t++)
            for (int e = 0; e < 4; e++) {
                acc_re[t][e] = 0.f;
                acc_im[t][e] = 0.f;
            }
        auto consume = [&](const unsigned char *buf) __attribute__((always_inline)) {
            switch (nrt) {
                case 4: consume_pairs_b3<L, 4>(buf, o_rb, o_cb, o_wb, l16, lk, acc_re, acc_im); break;
                case 3: consume_pairs_b3<L, 3>(buf, o_rb, o_cb, o_wb, l16, lk, acc_re, acc_im); break;
                case 2: consume_pairs_b3<L, 2>(buf, o_rb, o_cb, o_wb, l16, lk, acc_re, acc_im); break;
                case 1: consume_pairs_b3<L, 1>(buf, o_rb, o_cb, o_wb, l16, lk, acc_re, acc_im); break;
                default: break;
            }
        };
        auto run = [&](auto ky) {
            if (fetcher) {
                fetch(0);
                stash(0, decltype(ky)::value);
                fetch(1);
                stash(1, decltype(ky)::value);
            }
            __syncthreads();  // antenna table and the first two stages' sources ready
            produce(lds, 0, ky);
            __syncthreads();
            for (int stg = 0; stg < n_stage; stg++) {
                unsigned char *cur = lds + (stg & 1) * BUF;
                unsigned char *nxt = lds + ((stg + 1) & 1) * BUF;
                const bool more = stg + 1 < n_stage;
                if (fetcher && stg + 2 < n_stage) fetch(stg + 2);
                if (mult_first) consume(cur);
                if (more) produce(nxt, stg + 1, ky);
                if (!mult_first) consume(cur);
                // the sources of parity stg & 1 were last read by the producers of stage stg
                if (fetcher && stg + 2 < n_stage) stash(stg + 2, decltype(ky)::value);
                __syncthreads();
            }
        };
        if (kind_y)
            run(std::true_type{});
        else
            run(std::false_type{});

        int ld = Np;
        asm volatile("" : "+v"(ld));
        float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
        // product pr at antennas A of block I (rows) and B of block J (columns), A > B:
        //   X: V^pp at (2 A + pr, 2 B + pr);
        //   Y: pr = 0, V^10 at (2 A + 1, 2 B); pr = 1, V^01 at (2 A, 2 B + 1)
        const int row_off = kind_y ? 1 - pr : pr, col_off = kind_y ? pr : pr;
#pragma unroll
        for (int i = 0; i < kTI; i++)
#pragma unroll
            for (int j = 0; j < kTI; j++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int A = I * kST + 16 * (r0 + i) + 4 * lk + e, Bc = J * kST + 16 * (4 * ch + j) + l16;
                    if (i >= nrt || A >= a.n_ant || Bc >= a.n_ant) continue;
                    P[(int64_t)(2 * A + row_off) * ld + 2 * Bc + col_off] =
                        make_float2(acc_re[i * kTI + j][e], acc_im[i * kTI + j][e]);
                }
    }
}

// ---------------------------------------------------------------------------
// Scalar rows (one feed, one axis, one shared beam) in three blocks of 128
// (257..384 antennas).  Each item pairs one diagonal triangle with one full
// off-diagonal block that shares its rows, so every item stages two row blocks
// and the three items of an (instance, k-split) form 768 rows instead of the
// 1152 of one item per super-tile:
//   kind 0: V_10 and the triangle of block 0;  kind 1: V_21 and block 1;
//   kind 2: V_20 and block 2.
// LDS plane 0 holds the column block C, plane 1 the row block R (16 sources per
// stage).  Waves 0-3 take V_RC as four 64 x 64 wave tiles, multiply then form;
// waves 4-7 take the triangle as two-row sets {s, 7 - s} (nine tiles each),
// form then multiply.  With one beam, V_ab = sum_m |B_m|^2 F_a(m) conj(F_b(m)),
// so the rows are |B_m| F_a(m): a real scale instead of a complex product.
// ---------------------------------------------------------------------------
struct SclSrc {
    double x, y, z;  // s_hat
    float g, pad;    // |B| (0 past the split)
};

// SPS_: sources per stage, 16 or (BF16X3, the default there) 32: a deeper
// stage halves the barriers and the per-stage operand loads per source (3-5 %
// on the 350-antenna diffuse sky), the LDS holds 147 KB; the MFMAs accumulate
// in the same source order either way.
template <int PREC, int SQ_ROWS = 96, int SPS_ = 16>
__global__ void __launch_bounds__(512, 1) k_herk_blk3(FusedArgs a) {
    static_assert(SPS_ == 16 || (SPS_ == 32 && PREC == PB3), "16 sources per stage, or 32 on BF16X3");
    // 288- and 160-byte rows on BF16X3 (conflict-free operand reads), 144 on FP32
    typedef typename std::conditional<SPS_ == 32, GeomPair3,
                                      typename std::conditional<PREC == PB3, GeomCoh3, GeomCoh>::type>::type L;
    constexpr int RS = L::RS;
    constexpr int SPS = SPS_;
    constexpr int RSTEP = 512 / SPS;  // rows between a thread's rows
    constexpr int BUF = 2 * kST * RS;
    // SQ_ROWS: rows formed by the square waves of the 256 of a stage (the triangle
    // waves, with fewer products, form the rest); 96 by default, 64 and 128 as
    // tuning variants
    static_assert(SQ_ROWS % 32 == 0 && (2 * kST - SQ_ROWS) % 32 == 0, "32 rows per pass of a wave group");
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];
    __shared__ AntEntry tab[2 * kST];
    __shared__ SclSrc src[2][SPS];
    static_assert(2 * BUF + sizeof(tab) + sizeof(src) <= 160 * 1024, "LDS of one CU");

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const bool sq = wave < 4;
    const int l16 = lane & 15, lk = lane >> 4;
    const int Np = a.n_rows_pad;
    constexpr int n_kind = 3;
    const int total = a.work[a.n_inst] * n_kind;
    const int per_xcd = a.grid / 8;
    const int slot_x = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int mp = tid % (SPS / 2);
    // 16-source stages: 8 threads per row, rows permuted as in the two-block kernels
    const int a0 = SPS == 32    ? (sq ? tid / (SPS / 2) : SQ_ROWS + (tid - 256) / (SPS / 2))
                   : PREC == PB3 ? (sq ? wrow160(tid) : SQ_ROWS + wrow160(tid - 256))
                                 : (sq ? wrow(tid) : SQ_ROWS + wrow(tid - 256));
    const int sq_c0 = 4 * (wave & 1);
    const int tri_s = (wave - 4) & 3;

    for (int item = slot_x; item < total; item += a.grid) {
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.work[mid] * n_kind <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int inst = lo;
        const int local = item - a.work[inst] * n_kind;
        const int s = local / n_kind;
        const int kind = local % n_kind;
        const int R = kind == 0 ? 1 : 2, C = kind == 1 ? 1 : 0, T = kind;
        const int tri_o = (T == C ? 0 : 1) * kST;
        // Only the last block (2) can be short.  Its rows past the antennas are not
        // formed; the square waves split its row tiles evenly (waves 0, 1 the first
        // half, 2, 3 the rest), and a triangle wave drops the rows of its set that
        // lie wholly past them.
        const int n_r = a.n_ant - R * kST < kST ? a.n_ant - R * kST : kST;
        const int n_t = a.n_ant - T * kST < kST ? a.n_ant - T * kST : kST;
        const int nt_r = (n_r + 15) / 16, nt0 = (nt_r + 1) / 2, nt_t = (n_t + 15) / 16;
        const int sq_r0 = (wave >> 1) ? nt0 : 0, sq_nr = (wave >> 1) ? nt_r - nt0 : nt0;
        const int tri_nr = 7 - tri_s < nt_t ? 2 : tri_s < nt_t ? 1 : 0;
        const int tslot = inst / a.nfb;
        const int f = a.f0 + inst % a.nfb;
        const int64_t M = a.count[tslot];
        const int64_t ms_per_split = a.kcols[inst];
        const int64_t m_begin = (int64_t)s * ms_per_split;
        const int64_t m_end = m_begin + ms_per_split < M ? m_begin + ms_per_split : M;
        const int n_stage = (int)((m_end - m_begin + SPS - 1) / SPS);
        const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
        const float2 *Bm = (const float2 *)a.B + (int64_t)inst * a.ld_src;

        {
            const double nu_c = a.freqs[f] / kSpeedOfLight;
            for (int as = tid; as < 2 * kST; as += 512) {
                const int ant = (as < kST ? C : R) * kST + (as & (kST - 1));
                AntEntry e;
                if (ant < a.n_ant) {
                    e.ux = nu_c * a.antc[3 * ant];
                    e.uy = nu_c * a.antc[3 * ant + 1];
                    e.uz = nu_c * a.antc[3 * ant + 2];
                    e.b = 0;
                } else {
                    e.ux = e.uy = e.uz = 0.0;
                    e.b = -1;
                }
                e.pad = 0;
                tab[as] = e;
            }
        }

        // per-source direction and |B|, loaded one stage ahead by the first SPS lanes of wave 0
        const bool fetcher = tid < SPS;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        float2 fb = make_float2(0.f, 0.f);
        auto fetch = [&](int stage) {
            const int64_t m = m_begin + (int64_t)stage * SPS + tid;
            fx = fy = fz = 0.0;
            fb = make_float2(0.f, 0.f);
            if (stage < n_stage && m < m_end) {
                fx = sh[m];
                fy = sh[a.ld_src + m];
                fz = sh[2 * a.ld_src + m];
                fb = Bm[m];
            }
        };
        auto stash = [&](int stage) {
            SclSrc &e = src[stage & 1][tid];
            e.x = fx;
            e.y = fy;
            e.z = fz;
            e.g = sqrtf(fb.x * fb.x + fb.y * fb.y);
            e.pad = 0.f;
        };
        // rows a0 + RSTEP k (plane row >> 7) of this thread's two sources; rows of
        // block R past its antennas are skipped (never multiplied, or only into
        // outputs that are never stored)
        auto produce_n = [&](unsigned char *buf, int stage, auto na) __attribute__((always_inline)) {
            constexpr int NA = decltype(na)::value;
            SclSrc w[2];
            w[0] = src[stage & 1][2 * mp];
            w[1] = src[stage & 1][2 * mp + 1];
#pragma unroll
            for (int k = 0; k < NA; k++) {
                const int as = a0 + RSTEP * k;
                if (as >= kST + n_r) continue;
                const AntEntry e = tab[as];
                float vr[2], vi[2];
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const double p = e.ux * w[q].x + e.uy * w[q].y + e.uz * w[q].z;
                    const float r = (float)__builtin_amdgcn_fract(p);
                    vi[q] = w[q].g * __builtin_amdgcn_sinf(-r);
                    vr[q] = w[q].g * __builtin_amdgcn_cosf(-r);
                }
                if constexpr (PREC == PB3) {
                    uint32_t h0, l0, h1, l1;
                    split2(vr[0], vi[0], h0, l0);
                    split2(vr[1], vi[1], h1, l1);
                    unsigned char *rp = buf + as * RS + mp * 8;
                    *(uint2 *)rp = make_uint2(h0, h1);
                    *(uint2 *)(rp + L::PLANEB) = make_uint2(l0, l1);
                } else {
                    *(u32x4 *)(buf + as * RS + mp * 16) =
                        u32x4{__float_as_uint(vr[0]), __float_as_uint(vi[0]), __float_as_uint(vr[1]), __float_as_uint(vi[1])};
                }
            }
        };
        auto produce = [&](unsigned char *buf, int stage) __attribute__((always_inline)) {
            if (sq)
                produce_n(buf, stage, std::integral_constant<int, SQ_ROWS / RSTEP>{});
            else
                produce_n(buf, stage, std::integral_constant<int, (2 * kST - SQ_ROWS) / RSTEP>{});
        };

        f32x4 acc_re[16], acc_im[16];
        for (int t = 0; t < 16; t++)
            for (int e = 0; e < 4; e++) {
                acc_re[t][e] = 0.f;
                acc_im[t][e] = 0.f;
            }
        auto sq_n = [&](const unsigned char *buf, auto nr) __attribute__((always_inline)) {
            constexpr int NR = decltype(nr)::value;
            if constexpr (PREC == PB3)
                consume_sq_b3<L, 16, NR, kTI>(buf, 8 + sq_r0, sq_c0, l16, lk, acc_re, acc_im);
            else
                consume_sq_f32<L, 16, NR, kTI>(buf, 8 + sq_r0, sq_c0, l16, lk, acc_re, acc_im);
        };
        auto tri_n = [&](const unsigned char *buf, auto set) __attribute__((always_inline)) {
            typedef typename decltype(set)::type TS;
            if constexpr (PREC == PB3)
                consume_tri_b3<L, TS>(buf, tri_o, l16, lk, acc_re, acc_im);
            else
                consume_tri_f32<L, TS>(buf, tri_o, l16, lk, acc_re, acc_im);
        };
        auto consume = [&](const unsigned char *buf) __attribute__((always_inline)) {
            if (sq) {
                switch (sq_nr) {
                    case 4: sq_n(buf, std::integral_constant<int, 4>{}); break;
                    case 3: sq_n(buf, std::integral_constant<int, 3>{}); break;
                    case 2: sq_n(buf, std::integral_constant<int, 2>{}); break;
                    case 1: sq_n(buf, std::integral_constant<int, 1>{}); break;
                    default: break;
                }
            } else if (tri_nr == 2) {
                switch (tri_s) {
                    case 0: tri_n(buf, SetTag<TriPair<0>>{}); break;
                    case 1: tri_n(buf, SetTag<TriPair<1>>{}); break;
                    case 2: tri_n(buf, SetTag<TriPair<2>>{}); break;
                    default: tri_n(buf, SetTag<TriPair<3>>{}); break;
                }
            } else if (tri_nr == 1) {
                switch (tri_s) {
                    case 0: tri_n(buf, SetTag<TriSingle<0>>{}); break;
                    case 1: tri_n(buf, SetTag<TriSingle<1>>{}); break;
                    case 2: tri_n(buf, SetTag<TriSingle<2>>{}); break;
                    default: tri_n(buf, SetTag<TriSingle<3>>{}); break;
                }
            }
        };

        if (fetcher) {
            fetch(0);
            stash(0);
            fetch(1);
            stash(1);
        }
        __syncthreads();  // antenna table and the first two stages' sources ready
        produce(lds, 0);
        __syncthreads();
        for (int stg = 0; stg < n_stage; stg++) {
            unsigned char *cur = lds + (stg & 1) * BUF;
            unsigned char *nxt = lds + ((stg + 1) & 1) * BUF;
            const bool more = stg + 1 < n_stage;
            if (fetcher && stg + 2 < n_stage) fetch(stg + 2);
            if (sq) consume(cur);
            if (more) produce(nxt, stg + 1);
            if (!sq) consume(cur);
            // src[stg & 1] was last read by the producers of stage stg (one stage ago)
            if (fetcher && stg + 2 < n_stage) stash(stg + 2);
            __syncthreads();
        }

        int ld = Np;
        asm volatile("" : "+v"(ld));
        float2 *P = (float2 *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
        if (sq) {
#pragma unroll
            for (int i = 0; i < kTI; i++)
#pragma unroll
                for (int j = 0; j < kTI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int A = R * kST + 16 * (sq_r0 + i) + 4 * lk + e, Bc = C * kST + 16 * (sq_c0 + j) + l16;
                        if (i < sq_nr && A < a.n_ant && Bc < a.n_ant)
                            P[(int64_t)A * ld + Bc] = make_float2(acc_re[i * kTI + j][e], acc_im[i * kTI + j][e]);
                    }
        } else {
#pragma unroll
            for (int t = 0; t < 9; t++) {
                const int Rr = t <= tri_s ? tri_s : 7 - tri_s, Cc = t <= tri_s ? t : t - tri_s - 1;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int A = T * kST + 16 * Rr + 4 * lk + e, Bc = T * kST + 16 * Cc + l16;
                    if (A < a.n_ant && Bc < a.n_ant)
                        P[(int64_t)A * ld + Bc] = make_float2(acc_re[t][e], acc_im[t][e]);
                }
            }
        }
    }
}

template <int PREC, bool DIAG>
hipError_t launch_kind(const FusedArgs &a, hipStream_t s) {
    if (a.n_feed == 2 && a.n_ax == 2)
        k_herk_fused<PREC, 2, 2, DIAG><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_feed == 2)
        k_herk_fused<PREC, 2, 1, DIAG><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_ax == 2)
        k_herk_fused<PREC, 1, 2, DIAG><<<a.grid, 512, 0, s>>>(a);
    else
        k_herk_fused<PREC, 1, 1, DIAG><<<a.grid, 512, 0, s>>>(a);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_prec(const FusedArgs &a, hipStream_t s, int which) {
    hipError_t e = hipSuccess;
    if (which != FUSED_PAIRS) e = launch_kind<PREC, true>(a, s);
    if (e != hipSuccess || a.n_rows_pad <= kST || which == FUSED_FIRST)
        return e;  // a single row block has no off-diagonal tiles
    return launch_kind<PREC, false>(a, s);
}

}  // namespace

hipError_t launch_pair(const FusedArgs &a, hipStream_t s) {
    if (a.n_feed == 2 && a.n_ax == 2)
        k_herk_b3_pair<2, 2><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_feed == 2)
        k_herk_b3_pair<2, 1><<<a.grid, 512, 0, s>>>(a);
    else if (a.n_ax == 2)
        k_herk_b3_pair<1, 2><<<a.grid, 512, 0, s>>>(a);
    else
        k_herk_b3_pair<1, 1><<<a.grid, 512, 0, s>>>(a);
    return hipGetLastError();
}

int fused_path(int prec, int n_feed, int n_ax, int n_beam, int n_ant, int n_rows_pad) {
    if ((prec == PB3 || prec == P32) && n_feed == 2 && n_ax == 2 && n_beam == 1 && n_ant > kST / 2)
        return MATVIS_PATH_SOURCES;  // shared polarised beam: product over sources, blocks of 128 antennas
    if ((prec == PB3 || prec == P32) && n_feed == 1 && n_ax == 1 && n_beam == 1 && n_rows_pad == 3 * kST)
        return MATVIS_PATH_FUSED_BLOCKS;  // scalar rows in three blocks: items pairing a triangle and a block
    if (prec == PB3 && n_rows_pad == 2 * kST) return MATVIS_PATH_FUSED_ROWS;  // two row blocks: one item per split
    return MATVIS_PATH_FUSED;
}

bool fused_has_pairs(int prec, const FusedArgs &a) {
    const int path = fused_path(prec, a.n_feed, a.n_ax, a.n_beam, a.n_ant, a.n_rows_pad);
    if (path == MATVIS_PATH_SOURCES) return a.n_rows_pad > 2 * kST;
    if (path == MATVIS_PATH_FUSED) return a.n_rows_pad > kST;
    return false;
}

hipError_t launch_herk_fused(int prec, const FusedArgs &a, hipStream_t s, int which) {
    if (a.n_inst <= 0) return hipSuccess;
    const int path = fused_path(prec, a.n_feed, a.n_ax, a.n_beam, a.n_ant, a.n_rows_pad);
    const bool first = which != FUSED_PAIRS, pairs = which != FUSED_FIRST;
    const int split = a.tile & 15;  // rows per stage formed by the square waves, in units of 32 (0: default)
    if (path == MATVIS_PATH_SOURCES) {
        if (first) {
            // the full diagonal blocks, then a short last block (at most 96 antennas)
            const int nb = a.n_rows_pad / (2 * kST);
            const bool has_short = a.n_ant - (nb - 1) * kST <= 96;
            if (prec == PB3) {
                if (nb > 1 || !has_short) {
                    if (split == 2)
                        k_herk_coh<PB3, false, 64><<<a.grid, 512, 0, s>>>(a);
                    else
                        k_herk_coh<PB3, false, 96><<<a.grid, 512, 0, s>>>(a);
                }
                if (has_short) k_herk_coh<PB3, false, 96, true><<<a.grid, 512, 0, s>>>(a);
            } else {
                if (nb > 1 || !has_short) {
                    if (split == 2)
                        k_herk_coh<P32, false, 64><<<a.grid, 512, 0, s>>>(a);
                    else
                        k_herk_coh<P32, false, 96><<<a.grid, 512, 0, s>>>(a);
                }
                if (has_short) k_herk_coh<P32, false, 96, true><<<a.grid, 512, 0, s>>>(a);
            }
        }
        if (pairs && a.n_rows_pad > 2 * kST) {  // pairs of antenna blocks
            // bits 4-5 of the variant: 0 the one-sided-weight pair kernel (BF16X3), 1 the
            // two-sided one; FP32 always takes the latter
            if (prec == PB3 && ((a.tile >> 4) & 3) == 0)
                k_herk_pairs<<<a.grid, 512, 0, s>>>(a);
            else if (prec == PB3)
                k_herk_coh<PB3, true><<<a.grid, 512, 0, s>>>(a);
            else
                k_herk_coh<P32, true><<<a.grid, 512, 0, s>>>(a);
        }
        return hipGetLastError();
    }
    if (path == MATVIS_PATH_FUSED_ROWS) return first ? launch_pair(a, s) : hipSuccess;
    if (path == MATVIS_PATH_FUSED_BLOCKS) {
        if (!first) return hipSuccess;
        if (prec == PB3 && !(a.tile & 64)) {  // 32 sources per stage unless bit 6 asks for 16
            if (split == 2)
                k_herk_blk3<PB3, 64, 32><<<a.grid, 512, 0, s>>>(a);
            else if (split == 4)
                k_herk_blk3<PB3, 128, 32><<<a.grid, 512, 0, s>>>(a);
            else
                k_herk_blk3<PB3, 96, 32><<<a.grid, 512, 0, s>>>(a);
        } else if (prec == PB3) {
            if (split == 2)
                k_herk_blk3<PB3, 64><<<a.grid, 512, 0, s>>>(a);
            else if (split == 4)
                k_herk_blk3<PB3, 128><<<a.grid, 512, 0, s>>>(a);
            else
                k_herk_blk3<PB3, 96><<<a.grid, 512, 0, s>>>(a);
        } else {
            if (split == 2)
                k_herk_blk3<P32, 64><<<a.grid, 512, 0, s>>>(a);
            else if (split == 4)
                k_herk_blk3<P32, 128><<<a.grid, 512, 0, s>>>(a);
            else
                k_herk_blk3<P32, 96><<<a.grid, 512, 0, s>>>(a);
        }
        return hipGetLastError();
    }
    if (prec == P32) return launch_prec<P32>(a, s, which);
    if (prec == PB3) return launch_prec<PB3>(a, s, which);
    return hipErrorInvalidValue;
}

int herk_fused_occupancy(int prec) {
    int nb = 1;
    hipError_t e = prec == P32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk_fused<P32, 2, 2, false>, 512, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk_fused<PB3, 2, 2, false>, 512, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb < 1 ? 1 : nb;
}

}  // namespace mv
