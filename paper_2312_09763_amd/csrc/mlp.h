// Learned beam: a Fourier-feature MLP (az, za, nu) -> 2 x 2 complex Jones
// matrix, evaluated and trained by the kernels of kernels_mlp.hip.
//
// Inputs (u, v, w) = (az / 2 pi, za / (pi / 2), (nu - nu0) / (nu1 - nu0)).
// Parameter vector (FP32, the master copy), in this order:
//   Bff [kFreq][2]      Fourier frequencies (fixed; not trained).  Row j
//                        multiplies (u, v); the az entries are integers, so
//                        every feature is periodic in az.
//   W1 [kHid][2 kFreq], b1 [kHid]      features -> hidden 1
//   W2, W3, W4 [kHid][kHid], b2..b4    hidden l -> hidden l + 1
//   W5 [kNet][kHid], b5 [kNet]         hidden 4 -> coefficients g[8 o + k]
// Features: phi_j = sin(2 pi Bff_j . (u, v)), phi_{kFreq + j} = cos(...).
// Hidden layers use SiLU(z) = z / (1 + exp(-z)).  Output o (re, im of J[p][k],
// (p, k) row-major) is the Chebyshev series out_o = sum_k T_k(2 w - 1) g[8 o + k]
// of degree kBasis - 1: the network sees the direction only, so one
// evaluation per (source, time) serves every channel.
// The four hidden-layer products round both operands to bf16 and accumulate
// in FP32 on MFMA; biases, SiLU and the basis sums are FP32; the head is FP32
// in training and a hi / lo bf16 split (three products) in inference.
#pragma once

#include <cstdint>

#include "internal.h"

namespace mv {

constexpr int kFreq = 128;                    // Fourier frequencies (2 kFreq features)
constexpr int kFeat = 2 * kFreq;              // 256
constexpr int kHid = 128;                     // hidden width
constexpr int kOut = 8;                       // 2 x 2 complex outputs
constexpr int kBasis = 8;                     // Chebyshev terms per output
constexpr int kNet = kOut * kBasis;           // network outputs
constexpr int kBffCols = 2;                   // Fourier matrix columns (u, v)
constexpr int64_t kOffBff = 0;
constexpr int64_t kOffW1 = kOffBff + kFreq * kBffCols;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kHid * kFeat;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kHid * kHid;
constexpr int64_t kOffW4 = kOffB3 + kHid;
constexpr int64_t kOffB4 = kOffW4 + (int64_t)kHid * kHid;
constexpr int64_t kOffW5 = kOffB4 + kHid;
constexpr int64_t kOffB5 = kOffW5 + (int64_t)kNet * kHid;
constexpr int64_t kNParams = kOffB5 + kNet;   // 90944

// Host launchers (kernels_mlp.hip).  Row-major FP32 operands; every call is
// asynchronous on stream s and returns the launch status.
namespace mlp {
hipError_t features(const float *x, int64_t n, const float *P, float *phi, hipStream_t s);
// Z = A B^T + bias with A(m, k) = A[m sam + k sak], B(n, k) = B[n sbn + k sbk];
// H = SiLU(Z) when act = 1.  bf16 rounds both operands to bf16 first.  A plain
// product (no bias, no H) over a long k may split k through the workspace ws
// (ws_elems floats; NULL disables the split).
hipError_t gemm(bool bf16, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbn, int64_t sbk, int M,
                int N, int K, const float *bias, float *Z, float *H, int act, float *ws, int64_t ws_elems,
                hipStream_t s);
hipError_t silu_bwd(const float *dH, const float *Z, float *dZ, int64_t n, hipStream_t s);
// The basis sums and the squared error: out_o = sum_k T_k(2 x[m][2] - 1) net[m][8 o + k],
// loss = sum (out - y)^2 / (8 n), dnet[m][8 o + k] = T_k 2 (out_o - y_o) / (8 n).
hipError_t loss_grad(const float *net, const float *x, const float *y, int64_t n, float *dnet, float *part,
                     float *loss, hipStream_t s);
// db[c] = sum_m dZ[m][c] (fixed summation order) through the workspace ws
hipError_t colsum(const float *dZ, int64_t M, int N, float *db, float *ws, int64_t ws_elems, hipStream_t s);
hipError_t adam(float *p, const float *g, float *m1, float *m2, int64_t n, int64_t step, float lr, hipStream_t s);
hipError_t fill(float *out, int64_t n, float v, hipStream_t s);
hipError_t to_bf16(const float *in, __bf16 *out, int64_t n, hipStream_t s);
// bf16 W1..W4 (kWbElems values, 160 KB) in the inference kernel's LDS image:
// 1 KB MFMA A-operand blocks per (layer, 16-row tile, 32-deep k block), the
// columns of W2..W4 permuted to the accumulator order of the layer before;
// then the hi and lo bf16 parts of W5 in the same block form (kW5Elems, read
// from device memory by the head).  kImgElems values in all.
constexpr int64_t kWbElems = (int64_t)kHid * kFeat + 3 * (int64_t)kHid * kHid;
constexpr int64_t kW5Elems = 2 * (int64_t)kNet * kHid;
constexpr int64_t kImgElems = kWbElems + kW5Elems;
hipError_t pack_weights(const float *P, __bf16 *Wb, hipStream_t s);
hipError_t beam_samples(const void *grid, int n_feed, int n_ax, int n_za, int n_az, double dza, double daz,
                        int bicubic, const double *za, const double *az, const int32_t *chan, int64_t n, float *out,
                        const double *chan_freq, double nu0, double nu1, float *x, hipStream_t s);
hipError_t infer_plain(const float *P, const __bf16 *Wb, const float *x, int64_t n, float *out, hipStream_t s);
// Simulator mode: A of every instance of batch bt = sqrt(I) J (sqrt(I) = 1
// when idx is NULL), or J M for a polarised sky (pol: flux holds the Stokes
// planes stokes_stride apart, M of pol_sqrt; n_ax = 2), at the batch's
// visible sources, into beam slot `beam` of A [inst][n_beam][n_feed][n_ax][ld].
hipError_t infer_sim(const float *P, const __bf16 *Wb, double nu0, double nu1, const double *za_az,
                     const int32_t *count, const int32_t *idx, const double *flux, int64_t n_src, int pol,
                     int64_t stokes_stride, const double *freqs, int64_t ld_src, int64_t max_m, void *A, int n_feed,
                     int n_ax, int beam, int n_beam, const Batch &bt, hipStream_t s);
hipError_t gather_rows(const float *src, int width, const int32_t *perm, int64_t n, float *dst, hipStream_t s);
}  // namespace mlp

}  // namespace mv
