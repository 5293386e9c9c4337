// Alg. 2 step (v): V = Z Z^H (Eq. zz) for a batch of instances with uneven
// column counts, on MFMA.
//
// Real embedding.  With Z = Zr + i Zi,
//   Re V = Zr Zr^T + Zi Zi^T,   Im V = Zi Zr^T - Zr Zi^T,
// so each 16x16 output tile takes four real products per k-chunk (FP32 and
// FP64: v_mfma_{f32,f64}_16x16x4, one complex element per lane), or six bf16
// products on BF16X3 (v_mfma_f32_16x16x32_bf16: eight bf16 = four complex per
// lane, re/im interleaved; the imaginary operand W = (im, -re) is formed in
// registers by swapping the bf16 halves and flipping one sign bit, and
// Z Z^H ~ hi hi^H + hi lo^H + lo hi^H).
//
// Work decomposition.  Output rows are padded to Np, a multiple of the
// super-tile ST (128 on FP32/BF16X3, 64 on FP64).  A work item is
// (instance, k-split, lower super-tile (I >= J)).  A 256-thread workgroup
// stages the rows of I and J (only I on the diagonal) for KC = 16 complex
// columns at a time in LDS, with the next chunk prefetched into registers;
// its four waves own the 2 x 2 wave tiles of the super-tile (the wave above
// the diagonal of a diagonal super-tile idles).  Each item writes its
// partial tile to its own slot, so the later sum over k-splits runs in a
// fixed order and the result is bitwise reproducible.
//
// Scheduling.  The grid is persistent (a multiple of 8 workgroups); the
// per-instance item counts come from the device-side visible counts through
// a prefix array built by k_worklist, so no host synchronisation is needed.
// Workgroup b runs on XCD b % 8; consecutive items (the super-tiles of one
// k-split, which share Z rows) are mapped to workgroups of the same XCD so
// the shared rows hit the same L2.
#include "internal.h"

namespace mv {

namespace {

template <int PREC>
struct HT;
template <>
struct HT<P32> {
    static constexpr int ST = 128, KC = 16, EB = 8, PLANES = 1;
};
template <>
struct HT<P64> {
    static constexpr int ST = 64, KC = 16, EB = 16, PLANES = 1;
};
template <>
struct HT<PB3> {
    static constexpr int ST = 128, KC = 16, EB = 4, PLANES = 2;
};

// Stage geometry of a square ST_ tile computed by four waves (2 x 2 wave tiles).
template <int PREC, int ST_>
struct HG {
    typedef HT<PREC> T;
    static constexpr int ST = ST_, WT = ST_ / 2, KC = T::KC, EB = T::EB, PLANES = T::PLANES;
    static constexpr int ROWB = KC * EB * PLANES;  // bytes of one staged row
    static constexpr int RS = ROWB + 16;           // LDS row stride (16 B pad against bank conflicts)
    static constexpr int CPR = ROWB / 16;          // 16-byte chunks per row
    static constexpr int NLD = 2 * ST * CPR / 256; // chunks per thread per stage
    static constexpr int LDS = 2 * ST * RS;
    static constexpr int TI = WT / 16;             // 16x16 tiles per wave side
};
template <int PREC>
struct HD : HG<PREC, HT<PREC>::ST> {};

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Items of instance i: nsplit_i * n_st, with K_i = n_ax * visible count.
__device__ inline int64_t inst_k(const int32_t *count, int64_t fixed_k, int n_ax, int nfb, int i) {
    return count ? (int64_t)n_ax * count[i / nfb] : fixed_k;
}

// k-splits per instance and the item prefix.  nsplit_i starts at
// ceil(K_i / ksplit); with balancing, extra splits are spread over the
// instances until the total is a multiple of the persistent grid (capped by
// max_splits and by 64 columns per split), and each instance's splits are made
// equal: kcols_i = 64 ceil(K_i / (64 nsplit_i)).  Every workgroup then takes
// the same number of items of nearly the same size.
__global__ void __launch_bounds__(1024) k_worklist(const int32_t *count, int64_t fixed_k, int n_ax, int nfb, int n_inst,
                                                   int64_t ksplit, int n_st, int balance_grid, int max_splits,
                                                   int32_t *work, int32_t *nsplit, int32_t *kcols) {
    __shared__ int wtot[1024 / kWave];
    __shared__ int carry_s, total_s;
    if (threadIdx.x == 0) {
        carry_s = 0;
        total_s = 0;
    }
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int extra_all = 0;
    if (balance_grid > 0) {
        int part = 0;
        for (int i = threadIdx.x; i < n_inst; i += 1024) {
            const int64_t k = inst_k(count, fixed_k, n_ax, nfb, i);
            part += (int)((k + ksplit - 1) / ksplit);
        }
        atomicAdd(&total_s, part);
        __syncthreads();
        const int t = total_s;
        extra_all = (t + balance_grid - 1) / balance_grid * balance_grid - t;
    }
    for (int base = 0; base < n_inst; base += 1024) {
        int i = base + threadIdx.x;
        int v = 0;
        if (i < n_inst) {
            const int64_t k = inst_k(count, fixed_k, n_ax, nfb, i);
            int n = (int)((k + ksplit - 1) / ksplit);
            int64_t kc = ksplit;
            if (balance_grid > 0 && k > 0) {
                const int extra = extra_all / n_inst + (i < extra_all % n_inst ? 1 : 0);
                n = (int)min<int64_t>(min<int64_t>(n + extra, max_splits), (k + 63) / 64);
                kc = ((k + n - 1) / n + 63) / 64 * 64;
                n = (int)((k + kc - 1) / kc);
            }
            nsplit[i] = n;
            kcols[i] = (int32_t)kc;
            v = n * n_st;
        }
        int x = v;
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
            if (lane < 1024 / kWave) wtot[lane] = t;
        }
        __syncthreads();
        int carry = carry_s;
        if (i < n_inst) work[i] = carry + (w > 0 ? wtot[w - 1] : 0) + x - v;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + wtot[1024 / kWave - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) work[n_inst] = carry_s;
}

// W = (im, -re) for four packed bf16 complex values.
__device__ inline u32x4 bf16_rot(u32x4 v) {
    u32x4 r;
    for (int q = 0; q < 4; q++) r[q] = __builtin_amdgcn_alignbit(v[q], v[q], 16) ^ 0x80000000u;
    return r;
}

// One KC-deep stage of a WT x WT wave tile: rows arow.. of the staged A block
// against rows brow.. of the staged B block (both in LDS, row stride RS).
template <int PREC, typename D, typename Acc>
__device__ __forceinline__ void mma_stage(const unsigned char *lds, int arow, int brow, int l16, int lk, bool on_diag,
                                          Acc (&acc_re)[D::TI][D::TI], Acc (&acc_im)[D::TI][D::TI]) {
    constexpr int KC = D::KC, RS = D::RS, TI = D::TI;
    if constexpr (PREC == PB3) {
        u32x4 ah[TI], al[TI], bh[TI], bl[TI];
#pragma unroll
        for (int i = 0; i < TI; i++) {
            const unsigned char *p = lds + (arow + 16 * i + l16) * RS + lk * 16;
            ah[i] = *(const u32x4 *)p;
            al[i] = *(const u32x4 *)(p + KC * 4);
        }
#pragma unroll
        for (int j = 0; j < TI; j++) {
            const unsigned char *p = lds + (brow + 16 * j + l16) * RS + lk * 16;
            bh[j] = *(const u32x4 *)p;
            bl[j] = *(const u32x4 *)(p + KC * 4);
        }
#pragma unroll
        for (int i = 0; i < TI; i++) {
            const u32x4 wh = bf16_rot(ah[i]), wl = bf16_rot(al[i]);
            const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[i]);
            const bf16x8 Al = __builtin_bit_cast(bf16x8, al[i]);
            const bf16x8 Wh = __builtin_bit_cast(bf16x8, wh);
            const bf16x8 Wl = __builtin_bit_cast(bf16x8, wl);
#pragma unroll
            for (int j = 0; j < TI; j++) {
                const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]);
                const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[j]);
                acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, acc_re[i][j], 0, 0, 0);
                acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, acc_re[i][j], 0, 0, 0);
                acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acc_re[i][j], 0, 0, 0);
                acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wh, Bh, acc_im[i][j], 0, 0, 0);
                acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wh, Bl, acc_im[i][j], 0, 0, 0);
                acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl, Bh, acc_im[i][j], 0, 0, 0);
                // On the output diagonal the dropped lo lo^H term is a sum of
                // |lo|^2, a one-signed bias of relative size ~2^-16; add it
                // there (elsewhere it averages out and is left out).
                if (on_diag && i == j) {
                    acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bl, acc_re[i][j], 0, 0, 0);
                    acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wl, Bl, acc_im[i][j], 0, 0, 0);
                }
            }
        }
    } else {
        typedef typename std::conditional<PREC == P64, double2, float2>::type C;
        typedef typename std::conditional<PREC == P64, double, float>::type R;
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            C av[TI], bv[TI];
#pragma unroll
            for (int i = 0; i < TI; i++)
                av[i] = *(const C *)(lds + (arow + 16 * i + l16) * RS + (kk + lk) * D::EB);
#pragma unroll
            for (int j = 0; j < TI; j++)
                bv[j] = *(const C *)(lds + (brow + 16 * j + l16) * RS + (kk + lk) * D::EB);
#pragma unroll
            for (int i = 0; i < TI; i++) {
                const R nre = -av[i].x;
#pragma unroll
                for (int j = 0; j < TI; j++) {
                    if constexpr (PREC == P64) {
                        acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, acc_re[i][j], 0, 0, 0);
                        acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].y, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].x, acc_im[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nre, bv[j].y, acc_im[i][j], 0, 0, 0);
                    } else {
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, acc_re[i][j], 0, 0, 0);
                        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, acc_re[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].x, acc_im[i][j], 0, 0, 0);
                        acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nre, bv[j].y, acc_im[i][j], 0, 0, 0);
                    }
                }
            }
        }
    }
}

template <int PREC>
__global__ void __launch_bounds__(256, 2) k_herk(HerkArgs a) {
    typedef HD<PREC> D;
    constexpr int ST = D::ST, WT = D::WT, KC = D::KC, RS = D::RS, CPR = D::CPR, NLD = D::NLD, TI = D::TI;
    typedef typename std::conditional<PREC == P64, f64x4, f32x4>::type Acc;
    typedef typename std::conditional<PREC == P64, double2, float2>::type PartT;
    __shared__ __attribute__((aligned(16))) unsigned char lds[D::LDS];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    const int wr = wave >> 1, wc = wave & 1;
    const int Np = a.n_rows_pad;
    const int nb = Np / ST;
    const int n_st = nb * (nb + 1) / 2;
    const int total = a.work[a.n_inst];
    const int per_xcd = a.grid / 8;
    const int slot = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const char *zbase = (const char *)a.Z;
    const char *zlo = (const char *)a.Z_lo;
    const int64_t ldzb = a.ldz * D::EB;  // row stride in bytes of one plane

    for (int item = slot; item < total; item += a.grid) {
        // locate the instance: largest i with work[i] <= item
        int lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
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
        const bool diag = (I == J);
        const int64_t K = inst_k(a.count, a.fixed_k, a.n_ax, a.nfb, inst);
        const int64_t Kr = ((K + KC - 1) / KC) * KC;
        const int64_t kb = (int64_t)s * a.ksplit;
        const int64_t ke = kb + a.ksplit < Kr ? kb + a.ksplit : Kr;
        const int64_t ioff = (int64_t)inst * a.inst_stride * D::EB;

        Acc acc_re[TI][TI], acc_im[TI][TI];
        for (int i = 0; i < TI; i++)
            for (int j = 0; j < TI; j++)
                for (int e = 0; e < 4; e++) {
                    acc_re[i][j][e] = 0;
                    acc_im[i][j][e] = 0;
                }

        u32x4 pre[NLD];
        auto load = [&](int64_t k0) {
#pragma unroll
            for (int j = 0; j < NLD; j++) {
                if (diag && j >= NLD / 2) break;
                const int q = tid + 256 * j;
                const int lr = q / CPR, c = q % CPR;
                const int grow = lr < ST ? I * ST + lr : J * ST + (lr - ST);
                const char *src;
                if constexpr (D::PLANES == 2) {
                    const int half = CPR / 2;
                    src = (c < half ? zbase : zlo) + ioff + grow * ldzb + k0 * D::EB + (c % half) * 16;
                } else {
                    src = zbase + ioff + grow * ldzb + k0 * D::EB + c * 16;
                }
                pre[j] = *(const u32x4 *)src;
            }
        };
        auto store = [&]() {
#pragma unroll
            for (int j = 0; j < NLD; j++) {
                if (diag && j >= NLD / 2) break;
                const int q = tid + 256 * j;
                const int lr = q / CPR, c = q % CPR;
                *(u32x4 *)(lds + lr * RS + c * 16) = pre[j];
            }
        };

        const bool active = !(diag && wc > wr);
        const bool on_diag = diag && wc == wr;  // this wave's tiles (i, i) hold output diagonal entries
        const int arow = wr * WT;
        const int brow = (diag ? 0 : ST) + wc * WT;
        const int l16 = lane & 15, lk = lane >> 4;

        if (kb < ke) load(kb);
        for (int64_t k0 = kb; k0 < ke; k0 += KC) {
            __syncthreads();
            store();
            __syncthreads();
            if (k0 + KC < ke) load(k0 + KC);
            if (active) mma_stage<PREC, D>(lds, arow, brow, l16, lk, on_diag, acc_re, acc_im);
        }

        if (active) {
            // Accumulator layout of a 16x16 tile: lane l, register e holds column l % 16 of
            // row 4 (l / 16) + e for the f32 products, and of row 4 e + l / 16 for
            // v_mfma_f64_16x16x4f64.
            PartT *P = (PartT *)a.part + ((int64_t)inst * a.max_splits + s) * (int64_t)Np * Np;
            const int rb = I * ST + wr * WT;
            const int c0 = J * ST + wc * WT + l16;
#pragma unroll
            for (int i = 0; i < TI; i++)
#pragma unroll
                for (int j = 0; j < TI; j++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        PartT v;
                        v.x = acc_re[i][j][e];
                        v.y = acc_im[i][j][e];
                        const int row = rb + 16 * i + (PREC == P64 ? 4 * e + lk : 4 * lk + e);
                        P[(int64_t)row * Np + c0 + 16 * j] = v;
                    }
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

// Redundancy-aware product (App. A, Eq. Vpx): V'_x = A_x B_x^H with A_x, B_x
// gathered rows of Z.  One workgroup per (instance, ST x ST tile of a
// sub-matrix, k-split); the tile's rows are read through its two row lists
// straight from Z (a gather fused into the stage loads: no copy of A_x or
// B_x is formed), and the raw tile goes to its own partial slot.
template <int PREC, int STS>
__global__ void __launch_bounds__(256, 2) k_submat(SubmatArgs a) {
    typedef HG<PREC, STS> D;
    constexpr int ST = D::ST, WT = D::WT, KC = D::KC, RS = D::RS, CPR = D::CPR, NLD = D::NLD, TI = D::TI;
    typedef typename std::conditional<PREC == P64, f64x4, f32x4>::type Acc;
    typedef typename std::conditional<PREC == P64, double2, float2>::type PartT;
    __shared__ __attribute__((aligned(16))) unsigned char lds[D::LDS];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int wr = wave >> 1, wc = wave & 1, l16 = lane & 15, lk = lane >> 4;
    const int64_t item = blockIdx.x;
    const int s = (int)(item % a.max_splits);
    const int tile = (int)((item / a.max_splits) % a.n_tiles);
    const int inst = (int)(item / ((int64_t)a.max_splits * a.n_tiles));
    const int64_t K = inst_k(a.count, a.fixed_k, a.n_ax, a.nfb, inst);
    const int64_t Kr = ((K + KC - 1) / KC) * KC;
    const int64_t kb = (int64_t)s * a.ksplit;
    if (kb >= Kr) return;  // an empty k-split: the reduction sums only ceil(K / ksplit) of them
    const int64_t ke = kb + a.ksplit < Kr ? kb + a.ksplit : Kr;
    const int32_t *rows = a.rows + (int64_t)tile * 2 * ST;
    const char *zbase = (const char *)a.Z + (int64_t)inst * a.inst_stride * D::EB;
    const char *zlo = PREC == PB3 ? (const char *)a.Z_lo + (int64_t)inst * a.inst_stride * D::EB : nullptr;
    const int64_t ldzb = a.ldz * D::EB;

    Acc acc_re[TI][TI], acc_im[TI][TI];
    for (int i = 0; i < TI; i++)
        for (int j = 0; j < TI; j++)
            for (int e = 0; e < 4; e++) {
                acc_re[i][j][e] = 0;
                acc_im[i][j][e] = 0;
            }
    int grow[NLD];
#pragma unroll
    for (int j = 0; j < NLD; j++) {
        const int lr = (tid + 256 * j) / CPR;
        grow[j] = rows[lr];  // A rows for lr < ST, then B rows
    }
    u32x4 pre[NLD];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int j = 0; j < NLD; j++) {
            const int c = (tid + 256 * j) % CPR;
            pre[j] = u32x4{0u, 0u, 0u, 0u};
            if (grow[j] < 0) continue;
            if constexpr (D::PLANES == 2) {  // BF16X3: hi then lo plane of the staged row
                const int half = CPR / 2;
                pre[j] = *(const u32x4 *)((c < half ? zbase : zlo) + grow[j] * ldzb + k0 * D::EB + (c % half) * 16);
            } else {
                pre[j] = *(const u32x4 *)(zbase + grow[j] * ldzb + k0 * D::EB + c * 16);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < NLD; j++) {
            const int q = tid + 256 * j;
            *(u32x4 *)(lds + (q / CPR) * RS + (q % CPR) * 16) = pre[j];
        }
    };
    const int arow = wr * WT, brow = ST + wc * WT;
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += KC) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + KC < ke) load(k0 + KC);
        // BF16X3: any tile may hold an autocorrelation (a = b, p = q), where the
        // dropped lo lo^H term is a one-signed bias, so every tile takes it
        mma_stage<PREC, D>(lds, arow, brow, l16, lk, PREC == PB3, acc_re, acc_im);
    }
    PartT *P = (PartT *)a.part + (((int64_t)inst * a.max_splits + s) * a.n_tiles + tile) * ST * ST;
#pragma unroll
    for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TI; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                PartT v;
                v.x = acc_re[i][j][e];
                v.y = acc_im[i][j][e];
                const int r = arow + 16 * i + (PREC == P64 ? 4 * e + lk : 4 * lk + e);
                P[(int64_t)r * ST + wc * WT + 16 * j + l16] = v;
            }
}

// The same sub-matrix product with Z formed in the stages (FP32 and BF16X3):
// every staged element of the tile's A and B rows is
//   Z[(a, p), (m, k)] = B_{beam(a), p, k}(m) F_a(m),  F_a(m) = exp(-2 pi i nu x_a . s_m / c)
// (Eq. littlez with B = sqrt(I) A from the beam step), the phase range-reduced
// in FP64 and its sine and cosine taken on the hardware in revolutions, so Z
// never goes through device memory.  Thread t stages row t / 4 (A rows, then
// B rows) for four consecutive columns; the next stage's inputs are loaded
// before the current stage's products and turned into Z after them.
template <int PREC, int STS>
__global__ void __launch_bounds__(256, 2) k_submat_fused(SubmatArgs a) {
    typedef HG<PREC, STS> D;
    constexpr int ST = D::ST, WT = D::WT, KC = D::KC, RS = D::RS, TI = D::TI;
    static_assert(2 * ST * (KC / 4) == 256, "one thread per staged row and four columns");
    __shared__ __attribute__((aligned(16))) unsigned char lds[D::LDS];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int wr = wave >> 1, wc = wave & 1, l16 = lane & 15, lk = lane >> 4;
    const int64_t item = blockIdx.x;
    const int s = (int)(item % a.max_splits);
    const int tile = (int)((item / a.max_splits) % a.n_tiles);
    const int inst = (int)(item / ((int64_t)a.max_splits * a.n_tiles));
    const int64_t K = inst_k(a.count, a.fixed_k, a.n_ax, a.nfb, inst);
    const int64_t Kr = ((K + KC - 1) / KC) * KC;
    const int64_t kb = (int64_t)s * a.ksplit;
    if (kb >= Kr) return;  // an empty k-split: the reduction sums only ceil(K / ksplit) of them
    const int64_t ke = kb + a.ksplit < Kr ? kb + a.ksplit : Kr;
    const int nf = a.n_feed, nx = a.n_ax;
    const int r = tid / (KC / 4), cq = tid % (KC / 4);  // staged row, column group
    const int zrow = a.rows[(int64_t)tile * 2 * ST + r];  // a * n_feed + p, or -1
    const int ant = zrow < 0 ? 0 : zrow / nf, p = zrow < 0 ? 0 : zrow % nf;
    const int tslot = inst / a.nfb;
    const double nu_c = a.freqs[a.f0 + inst % a.nfb] / kSpeedOfLight;
    const double ux = nu_c * a.antc[3 * ant], uy = nu_c * a.antc[3 * ant + 1], uz = nu_c * a.antc[3 * ant + 2];
    const double *sh = a.s_hat + (int64_t)tslot * 3 * a.ld_src;
    const float2 *Bm = (const float2 *)a.B +
                       ((((int64_t)inst * a.n_beam + a.bidx[ant]) * nf + p) * nx) * a.ld_src;  // [k][m], stride ld_src

    typedef f32x4 Acc;
    Acc acc_re[TI][TI], acc_im[TI][TI];
    for (int i = 0; i < TI; i++)
        for (int j = 0; j < TI; j++)
            for (int e = 0; e < 4; e++) {
                acc_re[i][j][e] = 0.f;
                acc_im[i][j][e] = 0.f;
            }
    // inputs of this thread's four columns k0 + 4 cq + e: the source direction and its beam value
    double sx[4], sy[4], sz[4];
    float2 bv[4];
    float2 z[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int64_t col = k0 + 4 * cq + e;
            sx[e] = sy[e] = sz[e] = 0.0;
            bv[e] = make_float2(0.f, 0.f);
            if (zrow >= 0 && col < K) {
                const int64_t m = col / nx;
                sx[e] = sh[m];
                sy[e] = sh[a.ld_src + m];
                sz[e] = sh[2 * a.ld_src + m];
                bv[e] = Bm[(col % nx) * a.ld_src + m];
            }
        }
    };
    auto form = [&]() {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const double ph = ux * sx[e] + uy * sy[e] + uz * sz[e];
            const float rr = (float)__builtin_amdgcn_fract(ph);
            const float fi = __builtin_amdgcn_sinf(-rr), fr = __builtin_amdgcn_cosf(-rr);
            z[e] = make_float2(bv[e].x * fr - bv[e].y * fi, bv[e].x * fi + bv[e].y * fr);
        }
    };
    auto store = [&]() {
        unsigned char *row = lds + r * RS;
        if constexpr (PREC == PB3) {  // hi plane then lo plane, four bf16 pairs each
            uint32_t h[4], l[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const f32x2_t zz = {z[e].x, z[e].y};
                const bf16x2_t hh = __builtin_convertvector(zz, bf16x2_t);
                const f32x2_t rem = zz - __builtin_convertvector(hh, f32x2_t);
                const bf16x2_t ll = __builtin_convertvector(rem, bf16x2_t);
                h[e] = __builtin_bit_cast(uint32_t, hh);
                l[e] = __builtin_bit_cast(uint32_t, ll);
            }
            *(u32x4 *)(row + cq * 16) = u32x4{h[0], h[1], h[2], h[3]};
            *(u32x4 *)(row + KC * 4 + cq * 16) = u32x4{l[0], l[1], l[2], l[3]};
        } else {
            *(float4 *)(row + cq * 32) = make_float4(z[0].x, z[0].y, z[1].x, z[1].y);
            *(float4 *)(row + cq * 32 + 16) = make_float4(z[2].x, z[2].y, z[3].x, z[3].y);
        }
    };
    const int arow = wr * WT, brow = ST + wc * WT;
    load(kb);
    form();
    for (int64_t k0 = kb; k0 < ke; k0 += KC) {
        __syncthreads();
        store();
        __syncthreads();
        const bool more = k0 + KC < ke;
        if (more) load(k0 + KC);
        mma_stage<PREC, D>(lds, arow, brow, l16, lk, PREC == PB3, acc_re, acc_im);
        if (more) form();
    }
    float2 *P = (float2 *)a.part + (((int64_t)inst * a.max_splits + s) * a.n_tiles + tile) * ST * ST;
#pragma unroll
    for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TI; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int rr = arow + 16 * i + 4 * lk + e;
                P[(int64_t)rr * ST + wc * WT + 16 * j + l16] = make_float2(acc_re[i][j][e], acc_im[i][j][e]);
            }
}

// V of every requested pair: the k-split partials of its tile element summed in
// FP64 in split order, earlier source chunks carried in vacc.
template <int PREC>
__global__ void __launch_bounds__(256) k_submat_reduce(SubmatReduceArgs a) {
    typedef typename std::conditional<PREC == P64, double2, float2>::type C;
    const int nf = a.n_feed;
    const int64_t per_inst = (int64_t)a.n_pair * nf * nf;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= per_inst * a.n_inst) return;
    const int inst = (int)(gid / per_inst);
    const int64_t e = gid % per_inst;
    const int64_t K = inst_k(a.count, a.fixed_k, a.n_ax, a.nfb, inst);
    const int ns = (int)((K + a.ksplit - 1) / a.ksplit);
    const int32_t tile = a.loc[2 * e], off = a.loc[2 * e + 1];
    const int ST2 = a.st * a.st;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < ns; s++) {
        const C v = ((const C *)a.part)[(((int64_t)inst * a.max_splits + s) * a.n_tiles + tile) * ST2 + off];
        re += (double)v.x;
        im += (double)v.y;
    }
    double2 *acc = (double2 *)a.vacc + (int64_t)inst * per_inst + e;
    if (!a.first) {
        const double2 o = *acc;
        re += o.x;
        im += o.y;
    }
    if (!a.last) {
        *acc = make_double2(re, im);
        return;
    }
    const int t = a.bt.t0 + inst / a.bt.nfb, f = a.bt.f0 + inst % a.bt.nfb;
    C out;
    out.x = re;
    out.y = im;
    ((C *)a.out)[((int64_t)t * a.n_freq_total + f) * per_inst + e] = out;
}

// Fixed-order sum of the k-split partials, Hermitian fill and the write of the
// output layout, over 32 x 32 tiles of the lower triangle: partial rows are
// read coalesced, each lower element is summed once (in FP64, splits in
// order), and both it and its conjugate mirror above the diagonal are written,
// the mirror through an LDS transpose.  Earlier source chunks are carried in vacc at the
// lower positions only.
template <int PREC>
__global__ void __launch_bounds__(256) k_reduce_tiles(ReduceArgs a) {
    typedef typename std::conditional<PREC == P64, double2, float2>::type PartT;
    typedef typename std::conditional<PREC == P64, double2, float2>::type OutT;
    __shared__ double2 sm[32][33];
    const int inst = blockIdx.y;
    const int N = a.n_rows, Np = a.n_rows_pad, nf = a.n_feed, na = a.n_ant;
    // tile (R, C), R >= C, from the linear lower-triangle index
    int R = 0, t = blockIdx.x;
    while (t > R) {
        t -= R + 1;
        R++;
    }
    const int C = t;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t K = a.count ? (int64_t)a.n_ax * a.count[inst / a.nfb] : a.fixed_k;
    const int ns = a.nsplit ? a.nsplit[inst] : (int)((K + a.ksplit - 1) / a.ksplit);
    const PartT *P = (const PartT *)a.part + (int64_t)inst * a.max_splits * Np * Np;
    double2 *acc = a.vacc ? (double2 *)a.vacc + (int64_t)inst * N * N : nullptr;
    OutT *out = (OutT *)a.out;
    if (a.out_kind == 0) {
        const int tt = a.bt.t0 + inst / a.bt.nfb, f = a.bt.f0 + inst % a.bt.nfb;
        out += ((int64_t)tt * a.n_freq_total + f) * (int64_t)N * N;
    }
    auto out_index = [&](int r, int c) -> int64_t {
        if (a.out_kind != 0) return (int64_t)r * N + c;
        const int aa = r / nf, p = r % nf, b = c / nf, q = c % nf;
        return (((int64_t)aa * na + b) * nf + p) * nf + q;
    };
    for (int i = 0; i < 4; i++) {
        const int rl = ty + 8 * i, r = 32 * R + rl, c = 32 * C + tx;
        if (r >= N || c >= N || r < c) continue;
        const PartT *pp = P + (int64_t)r * Np + c;
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < ns; s++) {
            const PartT v = pp[(int64_t)s * Np * Np];
            sr += (double)v.x;
            si += (double)v.y;
        }
        if (r == c) si = 0.0;
        if (!a.first) {
            const double2 prev = acc[(int64_t)r * N + c];
            sr += prev.x;
            si += prev.y;
        }
        if (!a.last) {
            acc[(int64_t)r * N + c] = make_double2(sr, si);
            continue;
        }
        sm[rl][tx] = make_double2(sr, si);
        OutT v;
        v.x = sr;
        v.y = si;
        out[out_index(r, c)] = v;
    }
    if (!a.last) return;
    __syncthreads();
    // mirror: element (32 C + ty + 8 i, 32 R + tx) = conj(lower (32 R + tx, 32 C + ty + 8 i))
    for (int i = 0; i < 4; i++) {
        const int cl = ty + 8 * i, r = 32 * C + cl, c = 32 * R + tx;
        if (r >= N || c >= N || r >= c) continue;
        const double2 w = sm[tx][cl];
        OutT v;
        v.x = w.x;
        v.y = -w.y;
        out[out_index(r, c)] = v;
    }
}

}  // namespace

int herk_super_tile(int prec) { return prec == P64 ? HT<P64>::ST : HT<P32>::ST; }

hipError_t launch_submat(int prec, const SubmatArgs &a, hipStream_t s) {
    const int64_t items = (int64_t)a.n_inst * a.n_tiles * a.max_splits;
    if (items <= 0) return hipSuccess;
    if (prec == P64)
        k_submat<P64, kSubmatTile><<<(unsigned)items, 256, 0, s>>>(a);
    else if (prec == P32)
        k_submat<P32, kSubmatTile><<<(unsigned)items, 256, 0, s>>>(a);
    else if (prec == PB3)
        k_submat<PB3, kSubmatTile><<<(unsigned)items, 256, 0, s>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_submat_fused(int prec, const SubmatArgs &a, hipStream_t s) {
    const int64_t items = (int64_t)a.n_inst * a.n_tiles * a.max_splits;
    if (items <= 0) return hipSuccess;
    if (prec == P32)
        k_submat_fused<P32, kSubmatTile><<<(unsigned)items, 256, 0, s>>>(a);
    else if (prec == PB3)
        k_submat_fused<PB3, kSubmatTile><<<(unsigned)items, 256, 0, s>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_submat_reduce(int prec, const SubmatReduceArgs &a, hipStream_t s) {
    const int64_t n = (int64_t)a.n_inst * a.n_pair * a.n_feed * a.n_feed;
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (prec == P64)
        k_submat_reduce<P64><<<g, 256, 0, s>>>(a);
    else if (prec == P32 || prec == PB3)
        k_submat_reduce<P32><<<g, 256, 0, s>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int herk_occupancy(int prec) {
    int nb = 1;
    hipError_t e;
    if (prec == P64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk<P64>, 256, 0);
    else if (prec == P32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk<P32>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_herk<PB3>, 256, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return nb < 1 ? 1 : nb;
}

hipError_t launch_worklist(int prec, const HerkArgs &a, int unit, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    const int st = herk_super_tile(prec);
    const int nb = a.n_rows_pad / st;
    const int n_st = unit ? 1 : nb * (nb + 1) / 2;
    k_worklist<<<1, 1024, 0, s>>>(a.count, a.fixed_k, a.n_ax, a.nfb, a.n_inst, a.ksplit, n_st, a.balance_grid,
                                  a.max_splits, a.work, a.nsplit, a.kcols);
    return hipGetLastError();
}

hipError_t launch_herk(int prec, const HerkArgs &a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    if (prec == P64)
        k_herk<P64><<<a.grid, 256, 0, s>>>(a);
    else if (prec == P32)
        k_herk<P32><<<a.grid, 256, 0, s>>>(a);
    else
        k_herk<PB3><<<a.grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_reduce(int prec, const ReduceArgs &a, hipStream_t s) {
    if (a.n_inst <= 0 || a.n_rows <= 0) return hipSuccess;
    const int nt = (a.n_rows + 31) / 32;
    dim3 g((unsigned)(nt * (nt + 1) / 2), a.n_inst);
    if (prec == P64)
        k_reduce_tiles<P64><<<g, 256, 0, s>>>(a);
    else
        k_reduce_tiles<P32><<<g, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mv
