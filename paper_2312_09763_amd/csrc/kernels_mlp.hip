// Kernels of the learned beam (layout and network in mlp.h).
//
// Training runs on small row-major FP32 tensors: Fourier features, a strided
// MFMA GEMM with bias / SiLU epilogues (forward, and both backward products
// through stride choices), SiLU backward, the squared-error gradient, column
// sums for bias gradients, and Adam.  Products round their operands to bf16
// and accumulate in FP32 (v_mfma_f32_16x16x32_bf16), or stay in FP32
// (v_mfma_f32_16x16x4f32) in the FP32 check mode.
//
// Inference (k_mlp_infer) is one persistent launch: every workgroup holds
// the bf16 hidden weights in LDS and each wave runs the whole network on 64
// points at a time with the activations in registers, so only the inputs and
// the outputs touch HBM.  In the simulator it replaces beam interpolation:
// it reads the visible sources' (za, az) of one time, evaluates the network
// once, and writes B = sqrt(I) J of every channel of the batch (the
// Chebyshev sums of the frequency head) in the layout of the beam step.
#include <algorithm>

#include "beam_interp.h"
#include "mlp.h"

namespace mv {

namespace {

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }

// sin / cos of 2 pi r with the hardware units (argument in revolutions) after reduction
__device__ inline void sincos_rev(float r, float &s, float &c) {
    r -= rintf(r);
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}

// ---------------------------------------------------------------- features
__global__ void k_features(const float *__restrict__ x, int64_t n, const float *__restrict__ P,
                           float *__restrict__ phi) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * kFreq) return;
    const int64_t m = idx / kFreq;
    const int j = (int)(idx % kFreq);
    const float *b = P + kOffBff + kBffCols * j;
    const float arg = b[0] * x[3 * m] + b[1] * x[3 * m + 1];
    float s, c;
    sincos_rev(arg, s, c);
    phi[m * kFeat + j] = s;
    phi[m * kFeat + kFreq + j] = c;
}

// ---------------------------------------------------------------- GEMM
// C(m, n) = sum_k A(m, k) B(n, k) (+ bias[n]); A(m, k) = A[m sam + k sak],
// B(n, k) = B[n sbn + k sbk].  Z (if set) receives the pre-activation, H (if
// set) the activation (SiLU when act, else the same value).  64 x 64 output
// tile per 256-thread workgroup, 32-deep k steps through LDS; the staging
// loop walks whichever index has unit stride, so transposed operands are
// read coalesced.  Split-k: blockIdx.z takes k in [z kchunk, (z + 1) kchunk)
// and, when partial is set, stores its raw sum to partial[z][M][N] (summed in
// z order by k_sum_partials, so results do not depend on scheduling).
struct GemmArgs {
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbn, sbk;
    int M, N, K;
    const float *bias;
    float *Z;
    float *H;
    int act;
    int kchunk;
    float *partial;
};

template <bool BF16>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    constexpr int T = 64, KS = 32;
    constexpr int RSB = KS + 8;  // bf16 row stride (elements): 80 B, keeps 16-byte lane reads aligned
    constexpr int RSF = KS + 1;  // float row stride
    __shared__ __attribute__((aligned(16))) unsigned char smem[2 * T * (BF16 ? RSB * 2 : RSF * 4)];
    __bf16 *Ab = (__bf16 *)smem, *Bb = Ab + T * RSB;
    float *Af = (float *)smem, *Bf = Af + T * RSF;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int l16 = lane & 15, lk = lane >> 4;
    const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int kbeg = blockIdx.z * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
    const bool a_kfast = g.sak == 1, b_kfast = g.sbk == 1;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += KS) {
        for (int e = tid; e < T * KS; e += 256) {
            const int ra = a_kfast ? e / KS : e % T, ka = a_kfast ? e % KS : e / T;
            const int rb = b_kfast ? e / KS : e % T, kb = b_kfast ? e % KS : e / T;
            const int gm = m0 + ra, gka = k0 + ka, gn = n0 + rb, gkb = k0 + kb;
            const float va = (gm < g.M && gka < kend) ? g.A[gm * g.sam + gka * g.sak] : 0.f;
            const float vb = (gn < g.N && gkb < kend) ? g.B[gn * g.sbn + gkb * g.sbk] : 0.f;
            if (BF16) {
                Ab[ra * RSB + ka] = (__bf16)va;
                Bb[rb * RSB + kb] = (__bf16)vb;
            } else {
                Af[ra * RSF + ka] = va;
                Bf[rb * RSF + kb] = vb;
            }
        }
        __syncthreads();
        if (BF16) {
            bf16x8 a[2], b[2];
            for (int i = 0; i < 2; i++) a[i] = *(const bf16x8 *)(Ab + (wr + 16 * i + l16) * RSB + lk * 8);
            for (int j = 0; j < 2; j++) b[j] = *(const bf16x8 *)(Bb + (wc + 16 * j + l16) * RSB + lk * 8);
            for (int i = 0; i < 2; i++)
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
            for (int kk = 0; kk < KS; kk += 4) {
                float a[2], b[2];
                for (int i = 0; i < 2; i++) a[i] = Af[(wr + 16 * i + l16) * RSF + kk + lk];
                for (int j = 0; j < 2; j++) b[j] = Bf[(wc + 16 * j + l16) * RSF + kk + lk];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 2; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            for (int e = 0; e < 4; e++) {
                const int m = m0 + wr + 16 * i + 4 * lk + e, n = n0 + wc + 16 * j + l16;
                if (m >= g.M || n >= g.N) continue;
                if (g.partial) {
                    g.partial[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][e];
                    continue;
                }
                float v = acc[i][j][e] + (g.bias ? g.bias[n] : 0.f);
                if (g.Z) g.Z[(int64_t)m * g.N + n] = v;
                if (g.H) g.H[(int64_t)m * g.N + n] = g.act ? silu(v) : v;
            }
}

// ---------------------------------------------------------------- backward helpers
// dZ = dH * d SiLU/dz = dH * s (1 + z (1 - s)),  s = 1 / (1 + exp(-z))
__global__ void k_silu_bwd(const float *__restrict__ dH, const float *__restrict__ Z, float *__restrict__ dZ,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float z = Z[i];
    const float s = 1.0f / (1.0f + __expf(-z));
    dZ[i] = dH[i] * s * (1.0f + z * (1.0f - s));
}

// T_0..T_{kBasis-1} of the first kind at t (three-term recurrence)
__device__ inline void chebyshev(float t, float (&T)[kBasis]) {
    T[0] = 1.0f;
    T[1] = t;
#pragma unroll
    for (int k = 2; k < kBasis; k++) T[k] = 2.0f * t * T[k - 1] - T[k - 2];
}

// One thread per (row m, output o): out = sum_k T_k(2 w - 1) net[m][8 o + k]
// with w = x[m][2]; mean squared error over n x 8 outputs, dnet = T_k dOut with
// dOut = 2 (out - y) / (8 n); per-block partial sums of squares.
__global__ void __launch_bounds__(256) k_loss_grad(const float *__restrict__ net, const float *__restrict__ x,
                                                   const float *__restrict__ y, int64_t n, float *__restrict__ dnet,
                                                   float *__restrict__ part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.f;
    if (i < n * kOut) {
        const int64_t m = i / kOut;
        const int o = (int)(i % kOut);
        float T[kBasis];
        chebyshev(2.0f * x[3 * m + 2] - 1.0f, T);
        const float *g = net + m * kNet + o * kBasis;
        float out = 0.f;
#pragma unroll
        for (int k = 0; k < kBasis; k++) out += T[k] * g[k];
        const float d = out - y[i];
        const float dout = 2.0f * d / (float)(kOut * n);
        float *dg = dnet + m * kNet + o * kBasis;
#pragma unroll
        for (int k = 0; k < kBasis; k++) dg[k] = T[k] * dout;
        sq = d * d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Sequential sums (fixed order): out[0] = sum(part) / (8 n)
__global__ void k_finish_loss(const float *__restrict__ part, int nb, int64_t n, float *__restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += part[b];
    loss[0] = (float)(s / (double)(kOut * n));
}

// out[i] = sum_z part[z][i], z in order.
__global__ void k_sum_partials(const float *__restrict__ part, int nz, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < nz; z++) s += part[z * n + i];
    out[i] = s;
}

// Column sums of dZ [M][N] over row chunks of kColRows: part[chunk][c]; 64
// columns x 4 row lanes per workgroup, lanes combined in a fixed order.
constexpr int kColRows = 256;
__global__ void __launch_bounds__(256) k_colsum_part(const float *__restrict__ dZ, int64_t M, int N,
                                                     float *__restrict__ part) {
    __shared__ float red[4][64];
    const int cl = threadIdx.x % 64, rl = threadIdx.x / 64;
    const int c = blockIdx.x * 64 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * kColRows, r1 = min<int64_t>(M, r0 + kColRows);
    float s = 0.f;
    if (c < N)
        for (int64_t m = r0 + rl; m < r1; m += 4) s += dZ[m * N + c];
    red[rl][cl] = s;
    __syncthreads();
    if (rl == 0 && c < N) part[(int64_t)blockIdx.y * N + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

// Adam (Kingma & Ba 2015) on the trainable parameters (the Fourier matrix is fixed).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int64_t n, int64_t step, float lr, float b1, float b2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || i < kOffW1) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float ah = a / (1.0f - powf(b1, (float)step));
    const float bh = b / (1.0f - powf(b2, (float)step));
    p[i] -= lr * ah / (sqrtf(bh) + eps);
}

// dst[i][:] = src[perm[i]][:] (mini-batch assembly)
__global__ void k_gather_rows(const float *__restrict__ src, int width, const int32_t *__restrict__ perm, int64_t n,
                              float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * width) return;
    const int64_t r = i / width, c = i % width;
    dst[i] = src[(int64_t)perm[r] * width + c];
}

// out[i] = v (a kernel rather than a memset node, so the sequence may be captured into a graph)
__global__ void k_fill(float *__restrict__ out, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void k_to_bf16(const float *__restrict__ in, __bf16 *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (__bf16)in[i];
}

// ---------------------------------------------------------------- training samples
// out[i][8] = beam of channel chan[i] at (za[i], az[i]) from a complex64 grid
// [n_chan][n_feed][n_ax][n_za][n_az]; components beyond n_feed * n_ax are zero.
template <int MODE>
__global__ void k_beam_samples(const float2 *__restrict__ grid, int n_feed, int n_ax, int n_za, int n_az, double dza,
                               double daz, const double *__restrict__ za, const double *__restrict__ az,
                               const int32_t *__restrict__ chan, int64_t n, float *__restrict__ out,
                               const double *__restrict__ chan_freq, double nu0, double nu1, float *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (x) {
        // the network's normalised inputs, as the simulator forms them
        x[3 * i] = (float)(az[i] / (2.0 * M_PI));
        x[3 * i + 1] = (float)(za[i] / (0.5 * M_PI));
        x[3 * i + 2] = (float)((chan_freq[chan[i]] - nu0) / (nu1 - nu0));
    }
    const int ncomp = n_feed * n_ax;
    const int64_t plane = (int64_t)n_za * n_az;
    float2 v[4];
    for (int c = 0; c < 4; c++) v[c] = make_float2(0.f, 0.f);
    interp_point<float, MODE>(grid + (int64_t)chan[i] * ncomp * plane, plane, ncomp, n_za, n_az, dza, daz, za[i], az[i],
                              1.0f, v, 1);
    for (int c = 0; c < 4; c++) {
        out[i * kOut + 2 * c] = v[c].x;
        out[i * kOut + 2 * c + 1] = v[c].y;
    }
}

// ---------------------------------------------------------------- fused inference
// The whole network per 64 points in one wave, activations in registers.
// Layouts (v_mfma_f32_16x16x32_bf16, weights as the A operand, points as B):
// accumulator tile (h, pt) holds pre-activations of hidden units
// 16 h + 4 lk + e (e = 0..3) for point 16 pt + l16 in lane 16 lk + l16.  Two
// tiles (2 kb, 2 kb + 1) after SiLU are the next product's B operand for k
// block kb as they stand: lane (l16, lk) holds hidden units
// 32 kb + {4 lk .. 4 lk + 3, 16 + 4 lk .. 16 + 4 lk + 3}, and the LDS image
// of the next layer's weights permutes its columns the same way, so no
// activation ever leaves the registers.  The image of W1..W4 (160 KB, bf16,
// built by pack_weights) is resident in LDS for the whole persistent launch.
// The head takes hi and lo bf16 parts of W5 (from device memory) and of the
// last activations, three products accumulating in FP32 (the lo lo term,
// about 2^-16 of the product, is dropped): its accumulator tile (rt, pt)
// holds coefficient rows 16 rt + 4 lk + e = 8 o + k, i.e. output
// o = 2 rt + lk / 2 and terms k = 4 (lk & 1) + e, so a lane's partial basis
// sum plus its partner's (lane ^ 16) is output o.
constexpr int kBlk = 512;                                    // bf16 per 1 KB operand block
constexpr int kImgW1Blocks = (kHid / 16) * (kFeat / 32);     // 64: block h * 8 + kb
constexpr int kImgLayerBlocks = (kHid / 16) * (kHid / 32);   // 32 per layer 2..4: block h * 4 + kb
static_assert((int64_t)(kImgW1Blocks + 3 * kImgLayerBlocks) * kBlk == mlp::kWbElems, "image covers W1..W4");
constexpr int kImgW5Blocks = (kNet / 16) * (kHid / 32) * 2;  // 32: (row tile, k block, hi / lo)
static_assert((int64_t)kImgW5Blocks * kBlk == mlp::kW5Elems, "image covers W5 hi and lo");
constexpr int kIPts = 64;    // points per wave task
constexpr int kIWaves = 8;   // waves per workgroup (two per SIMD)

// column of W (row 16 h + l16) at element e of lane (l16, lk) in k block kb
__device__ __host__ inline int image_col(bool first, int kb, int lk, int e) {
    return first ? 32 * kb + 8 * lk + e : 32 * kb + (e < 4 ? 4 * lk + e : 12 + 4 * lk + e);
}

__global__ void k_pack_image(const float *__restrict__ P, __bf16 *__restrict__ img) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int)mlp::kImgElems) return;
    if (i >= (int)mlp::kWbElems) {
        // W5 hi / lo: block (rt * 4 + kb) * 2 + plane holds rows 16 rt + l16, the
        // columns of k block kb in the order of the hidden layers' operands
        const int j = i - (int)mlp::kWbElems;
        const int blk = j / kBlk, r = j % kBlk, L = r / 8, e = r % 8, l16 = L & 15, lk = L >> 4;
        const int plane = blk & 1, kb = (blk >> 1) & 3, rt = blk >> 3;
        const float w = P[kOffW5 + (int64_t)(16 * rt + l16) * kHid + image_col(false, kb, lk, e)];
        const __bf16 hi = (__bf16)w;
        img[i] = plane ? (__bf16)(w - (float)hi) : hi;
        return;
    }
    const int blk = i / kBlk, r = i % kBlk, L = r / 8, e = r % 8, l16 = L & 15, lk = L >> 4;
    int h, kb, K, col;
    const float *W;
    if (blk < kImgW1Blocks) {
        W = P + kOffW1;
        K = kFeat;
        h = blk / 8;
        kb = blk % 8;
        col = image_col(true, kb, lk, e);
    } else {
        const int l = (blk - kImgW1Blocks) / kImgLayerBlocks, b = (blk - kImgW1Blocks) % kImgLayerBlocks;
        W = P + (l == 0 ? kOffW2 : l == 1 ? kOffW3 : kOffW4);
        K = kHid;
        h = b / 4;
        kb = b % 4;
        col = image_col(false, kb, lk, e);
    }
    img[i] = (__bf16)W[(int64_t)(16 * h + l16) * K + col];
}

// SiLU with the hardware reciprocal (one rounding more than the division)
__device__ inline float silu_fast(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// operand block blk of the LDS image; loff = this lane's byte offset (lane * 16)
__device__ inline bf16x8 lds_block(const __bf16 *img, int blk, int loff) {
    return *(const bf16x8 *)((const char *)img + loff + blk * kBlk * 2);
}

// Hidden layer 2..4 (image blocks from blk0): out = SiLU(W in + b) as B operands.
__device__ inline void hidden_layer(const __bf16 *img, int blk0, const float *__restrict__ b, const bf16x8 (&in)[4][4],
                                    bf16x8 (&out)[4][4], int loff, int lk) {
#pragma unroll
    for (int hh = 0; hh < 2; hh++) {
        f32x4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const f32x4 bv = *(const f32x4 *)(b + 16 * (4 * hh + i) + 4 * lk);
#pragma unroll
            for (int pt = 0; pt < 4; pt++) acc[i][pt] = bv;
        }
#pragma unroll
        for (int kb = 0; kb < 4; kb++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const bf16x8 w = lds_block(img, blk0 + (4 * hh + i) * 4 + kb, loff);
#pragma unroll
                for (int pt = 0; pt < 4; pt++)
                    acc[i][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, in[kb][pt], acc[i][pt], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int pt = 0; pt < 4; pt++)
#pragma unroll
                for (int e = 0; e < 4; e++) out[2 * hh + i / 2][pt][4 * (i % 2) + e] = (__bf16)silu_fast(acc[i][pt][e]);
    }
}

struct InferArgs {
    const float *P;        // FP32 parameters (Fourier matrix, biases)
    const __bf16 *Wb;      // image: bf16 W1..W4 (copied to LDS), then W5 hi / lo
    double nu0, nu1;
    int64_t n_tasks;       // 64-point tasks
    int64_t tiles;         // simulator mode: tasks per time of the batch
    // plain mode: x [n][3] normalised inputs, out [n][8]
    const float *x;
    float *out;
    int64_t n;
    // simulator mode: visible sources of a batch
    const double *za_az;
    const int32_t *count;
    const int32_t *idx;
    const double *flux;
    int64_t n_src;
    int32_t pol;           // polarised sky: flux holds the Stokes planes stokes_stride apart
    int64_t stokes_stride;
    const double *freqs;
    int64_t ld_src;
    void *A;               // complex64 [inst][n_beam][n_feed][n_ax][ld_src] = sqrt(I) J (slot beam)
    int32_t n_feed, n_ax, beam, n_beam;
    Batch bt;
};

// J[p][0], J[p][1] (re, im each; p = lk, valid in lanes lk < 2) of point 16 pt + l16
// from the head accumulators and this lane's four basis values Tl[e] = T_{4 (lk & 1) + e}.
__device__ inline f32x4 basis_sum(const f32x4 (&D)[4][2], int pt, const float (&Tl)[4], int lk) {
    float s[4];
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        float v = Tl[0] * D[rt][pt][0];
#pragma unroll
        for (int e = 1; e < 4; e++) v += Tl[e] * D[rt][pt][e];
        s[rt] = v + __shfl_xor(v, 16);  // output 2 rt + lk / 2
    }
    const float a = (lk & 1) ? s[2] : s[0], b = (lk & 1) ? s[3] : s[1];  // re parts in lanes lk < 2
    return f32x4{a, __shfl_xor(a, 32), b, __shfl_xor(b, 32)};
}

template <bool SIM>
__global__ void __launch_bounds__(kIWaves * kWave) k_mlp_infer(InferArgs a) {
    __shared__ __attribute__((aligned(16))) __bf16 img[mlp::kWbElems];
    const int tid = threadIdx.x, lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int l16 = lane & 15, lk = lane >> 4;
    for (int i = tid; i < (int)(mlp::kWbElems / 8); i += kIWaves * kWave)
        ((u32x4 *)img)[i] = ((const u32x4 *)a.Wb)[i];
    __syncthreads();
    const int64_t nw = (int64_t)gridDim.x * kIWaves;
#pragma unroll 1
    for (int64_t t = (int64_t)blockIdx.x * kIWaves + wave; t < a.n_tasks; t += nw) {
        int slot = 0;
        int64_t m0, nrow;
        if (SIM) {  // 64 visible sources of one time of the batch, every channel
            slot = (int)(t / a.tiles);
            m0 = (t % a.tiles) * kIPts;
            nrow = a.count[slot];
            if (m0 >= nrow) continue;
        } else {
            m0 = t * kIPts;
            nrow = a.n;
        }
        // Parameters are re-read per task through L1: hoisted out of the loop
        // they would pin ~160 registers, so the pointer is made opaque here.
        const float *P = a.P;
        asm volatile("" : "+s"(P));
        // The same for the operand addresses: LDS blocks at loff + 1 KB blk, W5
        // blocks from w5: formed where they are read, not held across the loop.
        int loff = lane * 16;
        asm volatile("" : "+v"(loff));
        const __bf16 *w5 = a.Wb + mlp::kWbElems;
        asm volatile("" : "+s"(w5));
        // inputs of this lane's four points (16 pt + l16)
        float xu[4], xv[4], xw[4];
#pragma unroll
        for (int pt = 0; pt < 4; pt++) {
            const int64_t m = m0 + 16 * pt + l16;
            xu[pt] = xv[pt] = xw[pt] = 0.f;
            if (m < nrow) {
                if (SIM) {
                    const double za = a.za_az[(int64_t)slot * 2 * a.ld_src + m];
                    const double az = a.za_az[(int64_t)slot * 2 * a.ld_src + a.ld_src + m];
                    xu[pt] = (float)(az * (0.5 / M_PI));
                    xv[pt] = (float)(za * (2.0 / M_PI));
                } else {
                    xu[pt] = a.x[3 * m];
                    xv[pt] = a.x[3 * m + 1];
                    xw[pt] = a.x[3 * m + 2];
                }
            }
        }
        // layer 1: features formed per k block (sin in kb, cos in kb + 4)
        f32x4 acc1[8][4];
#pragma unroll
        for (int h = 0; h < 8; h++) {
            const f32x4 bv = *(const f32x4 *)(P + kOffB1 + 16 * h + 4 * lk);
#pragma unroll
            for (int pt = 0; pt < 4; pt++) acc1[h][pt] = bv;
        }
#pragma unroll 1
        for (int kb = 0; kb < 4; kb++) {
            float bf[16];
            const f32x4 *bsrc = (const f32x4 *)(P + kOffBff + kBffCols * (32 * kb + 8 * lk));
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const f32x4 v = bsrc[q];
                bf[4 * q] = v[0];
                bf[4 * q + 1] = v[1];
                bf[4 * q + 2] = v[2];
                bf[4 * q + 3] = v[3];
            }
            bf16x8 S[4], C[4];
#pragma unroll
            for (int pt = 0; pt < 4; pt++)
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    float s, c;
                    sincos_rev(bf[2 * e] * xu[pt] + bf[2 * e + 1] * xv[pt], s, c);
                    S[pt][e] = (__bf16)s;
                    C[pt][e] = (__bf16)c;
                }
#pragma unroll
            for (int h = 0; h < 8; h++) {
                const bf16x8 ws = lds_block(img, h * 8 + kb, loff), wc = lds_block(img, h * 8 + kb + 4, loff);
#pragma unroll
                for (int pt = 0; pt < 4; pt++) {
                    acc1[h][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ws, S[pt], acc1[h][pt], 0, 0, 0);
                    acc1[h][pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wc, C[pt], acc1[h][pt], 0, 0, 0);
                }
            }
        }
        bf16x8 hA[4][4], hB[4][4];
#pragma unroll
        for (int h = 0; h < 8; h++)
#pragma unroll
            for (int pt = 0; pt < 4; pt++)
#pragma unroll
                for (int e = 0; e < 4; e++) hA[h / 2][pt][4 * (h % 2) + e] = (__bf16)silu_fast(acc1[h][pt][e]);
        hidden_layer(img, kImgW1Blocks, P + kOffB2, hA, hB, loff, lk);
        hidden_layer(img, kImgW1Blocks + kImgLayerBlocks, P + kOffB3, hB, hA, loff, lk);
        // Layer 4, the head and the outputs for two point tiles at a time (points
        // 16 (2 pp + j) + l16, j < 2), which keeps the head's accumulators in registers.
        const int blk4 = kImgW1Blocks + 2 * kImgLayerBlocks;
#pragma unroll
        for (int pp = 0; pp < 2; pp++) {
            f32x4 acc[8][2];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const f32x4 bv = *(const f32x4 *)(P + kOffB4 + 16 * i + 4 * lk);
#pragma unroll
                for (int j = 0; j < 2; j++) acc[i][j] = bv;
            }
#pragma unroll
            for (int kb = 0; kb < 4; kb++)
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const bf16x8 w = lds_block(img, blk4 + i * 4 + kb, loff);
#pragma unroll
                    for (int j = 0; j < 2; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, hA[kb][2 * pp + j], acc[i][j], 0, 0, 0);
                }
            f32x4 D[4][2];
#pragma unroll
            for (int rt = 0; rt < 4; rt++) {
                const f32x4 b5 = *(const f32x4 *)(P + kOffB5 + 16 * rt + 4 * lk);
#pragma unroll
                for (int j = 0; j < 2; j++) D[rt][j] = b5;
            }
#pragma unroll
            for (int kb = 0; kb < 4; kb++) {  // head k block kb: unit tiles 2 kb, 2 kb + 1 after SiLU
                bf16x8 sh[2], sl[2];
#pragma unroll
                for (int j = 0; j < 2; j++)
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        const float v = silu_fast(acc[2 * kb + e / 4][j][e % 4]);
                        const __bf16 hi = (__bf16)v;
                        sh[j][e] = hi;
                        sl[j][e] = (__bf16)(v - (float)hi);
                    }
#pragma unroll
                for (int rt = 0; rt < 4; rt++) {
                    const bf16x8 wh = *(const bf16x8 *)(w5 + ((rt * 4 + kb) * 2) * kBlk + lane * 8);
                    const bf16x8 wl = *(const bf16x8 *)(w5 + ((rt * 4 + kb) * 2 + 1) * kBlk + lane * 8);
#pragma unroll
                    for (int j = 0; j < 2; j++) {
                        D[rt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, sh[j], D[rt][j], 0, 0, 0);
                        D[rt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, sl[j], D[rt][j], 0, 0, 0);
                        D[rt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, sh[j], D[rt][j], 0, 0, 0);
                    }
                }
            }
            if (!SIM) {
                // each point at its own frequency
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int pt = 2 * pp + j;
                    float T[kBasis], Tl[4];
                    chebyshev(2.0f * xw[2 * pp + j] - 1.0f, T);
#pragma unroll
                    for (int e = 0; e < 4; e++) Tl[e] = (lk & 1) ? T[4 + e] : T[e];
                    const f32x4 J = basis_sum(D, j, Tl, lk);
                    const int64_t m = m0 + 16 * pt + l16;
                    if (lk < 2 && m < nrow) *(f32x4 *)(a.out + m * kOut + 4 * lk) = J;
                }
                continue;
            }
            // every channel of the batch for this time
#pragma unroll 1
            for (int fi = 0; fi < a.bt.nfb; fi++) {
                const int inst = slot * a.bt.nfb + fi, f = a.bt.f0 + fi;
                float T[kBasis], Tl[4];
                chebyshev((float)(2.0 * (a.freqs[f] - a.nu0) / (a.nu1 - a.nu0) - 1.0), T);
#pragma unroll
                for (int e = 0; e < 4; e++) Tl[e] = (lk & 1) ? T[4 + e] : T[e];
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    f32x4 J = basis_sum(D, j, Tl, lk);  // (re, im) of J[lk][0], J[lk][1]
                    const int64_t m = m0 + 16 * (2 * pp + j) + l16;
                    if (lk >= 2 || m >= nrow) continue;
                    float sq = 1.0f;
                    if (a.idx) {
                        const int64_t o = (int64_t)f * a.n_src + a.idx[(int64_t)slot * a.ld_src + m];
                        if (a.pol) {
                            const PolSqrt pm = pol_sqrt(a.flux[o], a.flux[o + a.stokes_stride],
                                                        a.flux[o + 2 * a.stokes_stride],
                                                        a.flux[o + 3 * a.stokes_stride]);
                            float o0x, o0y, o1x, o1y;
                            apply_pol_sqrt<float>(pm, J[0], J[1], J[2], J[3], o0x, o0y, o1x, o1y);
                            J = f32x4{o0x, o0y, o1x, o1y};
                        } else {
                            sq = (float)sqrt(a.flux[o]);
                        }
                    }
                    // component (p, k) = (lk, cc) of the n_feed x n_ax Jones matrix
#pragma unroll
                    for (int cc = 0; cc < 2; cc++) {
                        if (lk >= a.n_feed || cc >= a.n_ax) continue;
                        float2 *dst = (float2 *)a.A +
                                      (((int64_t)inst * a.n_beam + a.beam) * a.n_feed * a.n_ax + lk * a.n_ax + cc) *
                                          a.ld_src + m;
                        *dst = make_float2(sq * J[2 * cc], sq * J[2 * cc + 1]);
                    }
                }
            }
        }
    }
}

int infer_grid(int64_t n_tasks) {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
            n_cu = 256;
    }
    return (int)std::min<int64_t>(n_cu, (n_tasks + kIWaves - 1) / kIWaves);
}

}  // namespace

// ---------------------------------------------------------------- host glue
namespace mlp {

hipError_t features(const float *x, int64_t n, const float *P, float *phi, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_features<<<(unsigned)((n * kFreq + 255) / 256), 256, 0, s>>>(x, n, P, phi);
    return hipGetLastError();
}

hipError_t gemm(bool bf16, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbn, int64_t sbk, int M,
                int N, int K, const float *bias, float *Z, float *H, int act, float *ws, int64_t ws_elems, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g{A, sam, sak, B, sbn, sbk, M, N, K, bias, Z, H, act, K, nullptr};
    dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
    // long reductions over few output tiles (the weight gradients): split k
    int nz = 1;
    const int tiles = (int)(grid.x * grid.y);
    if (ws && !bias && !H && !act && tiles < 128 && K >= 512) {
        nz = std::min<int>((K + 127) / 128, (256 + tiles - 1) / tiles);
        while (nz > 1 && (int64_t)nz * M * N > ws_elems) nz--;
    }
    if (nz > 1) {
        g.kchunk = (((K + nz - 1) / nz) + 31) / 32 * 32;
        nz = (K + g.kchunk - 1) / g.kchunk;
        g.partial = ws;
        grid.z = nz;
    }
    if (bf16)
        k_gemm<true><<<grid, 256, 0, s>>>(g);
    else
        k_gemm<false><<<grid, 256, 0, s>>>(g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nz == 1) return e;
    const int64_t n = (int64_t)M * N;
    k_sum_partials<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ws, nz, n, Z);
    return hipGetLastError();
}

hipError_t silu_bwd(const float *dH, const float *Z, float *dZ, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_silu_bwd<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dH, Z, dZ, n);
    return hipGetLastError();
}

hipError_t loss_grad(const float *net, const float *x, const float *y, int64_t n, float *dnet, float *part,
                     float *loss, hipStream_t s) {
    const int nb = (int)((n * kOut + 255) / 256);
    k_loss_grad<<<nb, 256, 0, s>>>(net, x, y, n, dnet, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish_loss<<<1, 64, 0, s>>>(part, nb, n, loss);
    return hipGetLastError();
}

hipError_t colsum(const float *dZ, int64_t M, int N, float *db, float *ws, int64_t ws_elems, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t nch = (M + kColRows - 1) / kColRows;
    if (nch * N > ws_elems) return hipErrorInvalidValue;
    k_colsum_part<<<dim3((unsigned)((N + 63) / 64), (unsigned)nch), 256, 0, s>>>(dZ, M, N, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_partials<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(ws, (int)nch, N, db);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m1, float *m2, int64_t n, int64_t step, float lr, hipStream_t s) {
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, g, m1, m2, n, step, lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t gather_rows(const float *src, int width, const int32_t *perm, int64_t n, float *dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_gather_rows<<<(unsigned)((n * width + 255) / 256), 256, 0, s>>>(src, width, perm, n, dst);
    return hipGetLastError();
}

hipError_t fill(float *out, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, v);
    return hipGetLastError();
}

hipError_t to_bf16(const float *in, __bf16 *out, int64_t n, hipStream_t s) {
    k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

hipError_t pack_weights(const float *P, __bf16 *Wb, hipStream_t s) {
    k_pack_image<<<(unsigned)((kImgElems + 255) / 256), 256, 0, s>>>(P, Wb);
    return hipGetLastError();
}

hipError_t beam_samples(const void *grid, int n_feed, int n_ax, int n_za, int n_az, double dza, double daz,
                        int bicubic, const double *za, const double *az, const int32_t *chan, int64_t n, float *out,
                        const double *chan_freq, double nu0, double nu1, float *x, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (bicubic)
        k_beam_samples<BICUBIC><<<nb, 256, 0, s>>>((const float2 *)grid, n_feed, n_ax, n_za, n_az, dza, daz, za, az,
                                                   chan, n, out, chan_freq, nu0, nu1, x);
    else
        k_beam_samples<BILINEAR><<<nb, 256, 0, s>>>((const float2 *)grid, n_feed, n_ax, n_za, n_az, dza, daz, za, az,
                                                    chan, n, out, chan_freq, nu0, nu1, x);
    return hipGetLastError();
}

hipError_t infer_plain(const float *P, const __bf16 *Wb, const float *x, int64_t n, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    InferArgs a{};
    a.P = P;
    a.Wb = Wb;
    a.x = x;
    a.out = out;
    a.n = n;
    a.n_tasks = (n + kIPts - 1) / kIPts;
    k_mlp_infer<false><<<infer_grid(a.n_tasks), kIWaves * kWave, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t infer_sim(const float *P, const __bf16 *Wb, double nu0, double nu1, const double *za_az,
                     const int32_t *count, const int32_t *idx, const double *flux, int64_t n_src, int pol,
                     int64_t stokes_stride, const double *freqs, int64_t ld_src, int64_t max_m, void *A, int n_feed,
                     int n_ax, int beam, int n_beam, const Batch &bt, hipStream_t s) {
    if (bt.n_inst <= 0 || max_m <= 0) return hipSuccess;
    if (n_feed > 2 || n_ax > 2) return hipErrorInvalidValue;
    InferArgs a{};
    a.P = P;
    a.Wb = Wb;
    a.nu0 = nu0;
    a.nu1 = nu1;
    a.za_az = za_az;
    a.count = count;
    a.idx = idx;
    a.flux = flux;
    a.n_src = n_src;
    a.pol = pol;
    a.stokes_stride = stokes_stride;
    a.freqs = freqs;
    a.ld_src = ld_src;
    a.A = A;
    a.n_feed = n_feed;
    a.n_ax = n_ax;
    a.beam = beam;
    a.n_beam = n_beam;
    a.bt = bt;
    a.tiles = (max_m + kIPts - 1) / kIPts;
    a.n_tasks = a.tiles * bt.ntb;  // one task per 64 sources of one time: every channel of the batch
    k_mlp_infer<true><<<infer_grid(a.n_tasks), kIWaves * kWave, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mlp

}  // namespace mv
