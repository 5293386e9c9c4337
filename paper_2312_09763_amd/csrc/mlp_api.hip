// Host side of the learned beam (include/matvis.h, "Learned beam").
// Forward and backward passes are chains of the kernels in kernels_mlp.hip;
// the training loop is native and only synchronises once per epoch to read
// the loss.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <numeric>
#include <random>
#include <vector>

#include "matvis.h"
#include "internal.h"
#include "mlp.h"

using namespace mv;

namespace {

#define CK(expr)                                       \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) {                        \
            (void)hipGetLastError();                   \
            fprintf(stderr, "%s: %s\n", #expr, hipGetErrorString(_e)); \
            return MATVIS_EHIP;                        \
        }                                              \
    } while (0)

// Activation workspace for n rows: buffer sizes in floats, in the order the
// workspace holds them.  alloc() gives each its own device allocation; bind()
// carves them, 256-byte aligned, out of one caller-provided block of
// Work::floats_for(rows) floats.
struct Work {
    int64_t n = 0;
    float *phi = nullptr, *Z[4] = {}, *H[4] = {}, *out = nullptr, *dout = nullptr, *dH = nullptr, *dZ = nullptr,
          *part = nullptr, *ws = nullptr;
    int64_t ws_elems = 0;  // split-k partial products and column-sum partials
    std::vector<void *> allocs;
    static int64_t ws_for(int64_t rows) { return std::max<int64_t>(384 * 4096, (rows + 255) / 256 * kHid); }
    // the (pointer, size) list in workspace order
    template <typename F>
    static hipError_t each(int64_t rows, float **phi, float **Z, float **H, float **out, float **dout, float **dH,
                           float **dZ, float **part, float **ws, F &&one) {
        hipError_t e = one(phi, rows * kFeat);
        for (int l = 0; l < 4 && e == hipSuccess; l++) e = one(&Z[l], rows * kHid);
        for (int l = 0; l < 4 && e == hipSuccess; l++) e = one(&H[l], rows * kHid);
        if (e == hipSuccess) e = one(out, rows * kNet);   // network outputs (basis coefficients)
        if (e == hipSuccess) e = one(dout, rows * kNet);
        if (e == hipSuccess) e = one(dH, rows * kHid);
        if (e == hipSuccess) e = one(dZ, rows * kHid);
        if (e == hipSuccess) e = one(part, (rows * kOut + 255) / 256 + 1);
        if (e == hipSuccess) e = one(ws, ws_for(rows));
        return e;
    }
    static constexpr int64_t kAlign = 64;  // floats (256 bytes)
    static int64_t round_a(int64_t c) { return (std::max<int64_t>(c, 1) + kAlign - 1) / kAlign * kAlign; }
    static int64_t floats_for(int64_t rows) {
        int64_t total = 0;
        float *dummy[16] = {};
        (void)each(rows, &dummy[0], &dummy[1], &dummy[5], &dummy[9], &dummy[10], &dummy[11], &dummy[12], &dummy[13],
                   &dummy[14], [&](float **, int64_t count) {
                 total += round_a(count);
                 return hipSuccess;
             });
        return total;
    }
    hipError_t alloc(int64_t rows) {
        n = rows;
        ws_elems = ws_for(rows);
        return each(rows, &phi, Z, H, &out, &dout, &dH, &dZ, &part, &ws, [&](float **p, int64_t count) {
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, sizeof(float) * std::max<int64_t>(count, 1));
            if (e == hipSuccess) {
                allocs.push_back(q);
                *p = (float *)q;
            }
            return e;
        });
    }
    // no allocation: the buffers are consecutive pieces of base[0 .. floats_for(rows))
    void bind(float *base, int64_t rows) {
        n = rows;
        ws_elems = ws_for(rows);
        int64_t off = 0;
        (void)each(rows, &phi, Z, H, &out, &dout, &dH, &dZ, &part, &ws, [&](float **p, int64_t count) {
            *p = base + off;
            off += round_a(count);
            return hipSuccess;
        });
    }
    ~Work() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

// Forward + backward of the squared error for w.n rows of (x, y).
hipError_t loss_grad_impl(const float *P, const float *x, const float *y, bool bf16, float *grad, float *loss, Work &w,
                          hipStream_t s) {
    const int64_t n = w.n;
    const int ni = (int)n;
    hipError_t e;
#define RET(expr)                      \
    if ((e = (expr)) != hipSuccess) return e
    RET(mlp::features(x, n, P, w.phi, s));
    RET(mlp::gemm(bf16, w.phi, kFeat, 1, P + kOffW1, kFeat, 1, ni, kHid, kFeat, P + kOffB1, w.Z[0], w.H[0], 1,
                  w.ws, w.ws_elems, s));
    const int64_t offW[3] = {kOffW2, kOffW3, kOffW4}, offB[3] = {kOffB2, kOffB3, kOffB4};
    for (int l = 1; l < 4; l++)
        RET(mlp::gemm(bf16, w.H[l - 1], kHid, 1, P + offW[l - 1], kHid, 1, ni, kHid, kHid, P + offB[l - 1], w.Z[l],
                      w.H[l], 1, w.ws, w.ws_elems, s));
    // the linear head in FP32 (inference splits it hi / lo), then the Chebyshev
    // sums of the frequency head and the squared error
    RET(mlp::gemm(false, w.H[3], kHid, 1, P + kOffW5, kHid, 1, ni, kNet, kHid, P + kOffB5, w.out, nullptr, 0,
                  w.ws, w.ws_elems, s));
    RET(mlp::loss_grad(w.out, x, y, n, w.dout, w.part, loss, s));
    RET(mlp::fill(grad, kOffW1, 0.f, s));  // the Fourier matrix is not trained
    // output layer
    RET(mlp::gemm(false, w.dout, 1, kNet, w.H[3], 1, kHid, kNet, kHid, ni, nullptr, grad + kOffW5, nullptr, 0,
                  w.ws, w.ws_elems, s));
    RET(mlp::colsum(w.dout, n, kNet, grad + kOffB5, w.ws, w.ws_elems, s));
    RET(mlp::gemm(false, w.dout, kNet, 1, P + kOffW5, 1, kHid, ni, kHid, kNet, nullptr, w.dH, nullptr, 0,
                  w.ws, w.ws_elems, s));
    // hidden layers 4..2
    const int64_t gW[4] = {kOffW1, kOffW2, kOffW3, kOffW4}, gB[4] = {kOffB1, kOffB2, kOffB3, kOffB4};
    for (int l = 3; l >= 1; l--) {
        RET(mlp::silu_bwd(w.dH, w.Z[l], w.dZ, n * kHid, s));
        RET(mlp::gemm(bf16, w.dZ, 1, kHid, w.H[l - 1], 1, kHid, kHid, kHid, ni, nullptr, grad + gW[l], nullptr, 0,
                      w.ws, w.ws_elems, s));
        RET(mlp::colsum(w.dZ, n, kHid, grad + gB[l], w.ws, w.ws_elems, s));
        RET(mlp::gemm(bf16, w.dZ, kHid, 1, P + gW[l], 1, kHid, ni, kHid, kHid, nullptr, w.dH, nullptr, 0,
                      w.ws, w.ws_elems, s));
    }
    RET(mlp::silu_bwd(w.dH, w.Z[0], w.dZ, n * kHid, s));
    RET(mlp::gemm(bf16, w.dZ, 1, kHid, w.phi, 1, kFeat, kHid, kFeat, ni, nullptr, grad + kOffW1, nullptr, 0,
                  w.ws, w.ws_elems, s));
    RET(mlp::colsum(w.dZ, n, kHid, grad + kOffB1, w.ws, w.ws_elems, s));
#undef RET
    return hipSuccess;
}

}  // namespace

// ---- The allocation-free loss / gradient (matvis_mlp_loss_grad_noalloc) ----
// Its workspace is one file-scope device array of kNoAllocRows rows' worth of
// activations (33.6 MB), which every GPU the library runs on holds until the
// process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept in noalloc_ptr.
static constexpr int64_t kNoAllocRows = 4096;
static constexpr int64_t kNoAllocFloats = 8388800;  // Work::floats_for(kNoAllocRows), checked below
static __device__ __align__(256) float scratch[kNoAllocFloats];

static constexpr int kMaxDevices = 64;
static std::mutex noalloc_mu;
static float *noalloc_ptr[kMaxDevices] = {};

static hipError_t noalloc_scratch(float **p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        noalloc_ptr[dev] = (float *)q;
    }
    *p = noalloc_ptr[dev];
    return hipSuccess;
}

extern "C" {

matvis_status matvis_mlp_forward(const float *params, const float *x, int64_t n, float *out, void *stream) {
    if (!params || (n > 0 && (!x || !out)) || n < 0) return MATVIS_EINVAL;
    if ((uintptr_t)params % 16 || (uintptr_t)out % 16) return MATVIS_EINVAL;  // read / written as float4
    if (n == 0) return MATVIS_OK;
    hipStream_t s = (hipStream_t)stream;
    __bf16 *wb = nullptr;
    CK(hipMalloc(&wb, sizeof(__bf16) * mlp::kImgElems));
    hipError_t e = mlp::pack_weights(params, wb, s);
    if (e == hipSuccess) e = mlp::infer_plain(params, wb, x, n, out, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(wb);
    CK(e);
    return MATVIS_OK;
}

matvis_status matvis_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t n, int32_t fp32_math,
                                   float *grad, float *loss, void *stream) {
    if (!params || !x || !y || !grad || !loss || n <= 0 || n > (1 << 24)) return MATVIS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Work w;
    CK(w.alloc(n));
    CK(loss_grad_impl(params, x, y, !fp32_math, grad, loss, w, s));
    CK(hipStreamSynchronize(s));
    return MATVIS_OK;
}

matvis_status matvis_mlp_loss_grad_noalloc(const float *params, const float *x, const float *y, int64_t n,
                                           int32_t fp32_math, float *grad, float *loss, void *stream) {
    if (!params || !x || !y || !grad || !loss || n <= 0) return MATVIS_EINVAL;
    if (n > kNoAllocRows) {
        fprintf(stderr,
                "matvis_mlp_loss_grad_noalloc: n = %lld rows exceeds the static workspace of %lld rows "
                "(use matvis_mlp_loss_grad)\n",
                (long long)n, (long long)kNoAllocRows);
        return MATVIS_EINVAL;
    }
    if (Work::floats_for(kNoAllocRows) != kNoAllocFloats) {  // layout and array size out of step
        fprintf(stderr, "matvis_mlp_loss_grad_noalloc: workspace layout needs %lld floats, array holds %lld\n",
                (long long)Work::floats_for(kNoAllocRows), (long long)kNoAllocFloats);
        return MATVIS_EUNSUPPORTED;
    }
    float *base = nullptr;
    CK(noalloc_scratch(&base));
    Work w;
    w.bind(base, n);
    CK(loss_grad_impl(params, x, y, !fp32_math, grad, loss, w, (hipStream_t)stream));
    return MATVIS_OK;
}

matvis_status matvis_mlp_adam(float *params, const float *grad, float *m1, float *m2, int64_t step, float lr,
                              void *stream) {
    if (!params || !grad || !m1 || !m2 || step < 1) return MATVIS_EINVAL;
    CK(mlp::adam(params, grad, m1, m2, kNParams, step, lr, (hipStream_t)stream));
    return MATVIS_OK;
}

matvis_status matvis_beam_samples(const void *grid, int32_t n_chan, int32_t n_feed, int32_t n_ax, int32_t n_za,
                                  int32_t n_az, double dza_rad, double daz_rad, int32_t bicubic, const double *za,
                                  const double *az, const int32_t *chan, int64_t n, float *out,
                                  const double *chan_freq_hz, double nu_min_hz, double nu_max_hz, float *x,
                                  void *stream) {
    if (!grid || (n > 0 && (!za || !az || !chan || !out)) || n < 0) return MATVIS_EINVAL;
    if (x && (!chan_freq_hz || !std::isfinite(nu_min_hz) || !std::isfinite(nu_max_hz) || !(nu_max_hz > nu_min_hz)))
        return MATVIS_EINVAL;
    if (n_chan <= 0 || n_feed < 1 || n_feed > 2 || n_ax < 1 || n_ax > 2 || n_za < 3 || n_az < 3) return MATVIS_EINVAL;
    if (!(dza_rad > 0) || !(daz_rad > 0)) return MATVIS_EINVAL;
    // validate the channel indices here so that no kernel reads outside the grid
    std::vector<int32_t> h((size_t)n);
    CK(hipMemcpy(h.data(), chan, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int32_t c : h)
        if (c < 0 || c >= n_chan) return MATVIS_EINVAL;
    CK(mlp::beam_samples(grid, n_feed, n_ax, n_za, n_az, dza_rad, daz_rad, bicubic, za, az, chan, n, out,
                         chan_freq_hz, nu_min_hz, nu_max_hz, x, (hipStream_t)stream));
    return MATVIS_OK;
}

matvis_status matvis_train_surrogate(float *params, const float *x, const float *y, int64_t n, int32_t batch,
                                     int32_t epochs, float lr0, float lr1, uint64_t seed, int32_t fp32_math,
                                     float *loss_history, void *stream) {
    if (!params || !x || !y || n <= 0 || n > (1 << 30) || batch <= 0 || batch > (1 << 24) || epochs <= 0 ||
        !(lr0 > 0) || !(lr1 > 0))
        return MATVIS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t bsz = std::min<int64_t>(batch, n);
    Work w;
    CK(w.alloc(bsz));
    float *grad = nullptr, *m1 = nullptr, *m2 = nullptr, *xb = nullptr, *yb = nullptr, *lossd = nullptr;
    int32_t *perm_d = nullptr;
    std::vector<void *> allocs;
    auto al = [&](void **p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) allocs.push_back(*p);
        return e;
    };
    hipError_t e = al((void **)&grad, sizeof(float) * kNParams);
    if (e == hipSuccess) e = al((void **)&m1, sizeof(float) * kNParams);
    if (e == hipSuccess) e = al((void **)&m2, sizeof(float) * kNParams);
    if (e == hipSuccess) e = al((void **)&xb, sizeof(float) * bsz * 3);
    if (e == hipSuccess) e = al((void **)&yb, sizeof(float) * bsz * kOut);
    if (e == hipSuccess) e = al((void **)&lossd, sizeof(float) * 4096);
    if (e == hipSuccess) e = al((void **)&perm_d, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMemsetAsync(m1, 0, sizeof(float) * kNParams, s);
    if (e == hipSuccess) e = hipMemsetAsync(m2, 0, sizeof(float) * kNParams, s);
    std::vector<int32_t> perm((size_t)n);
    std::iota(perm.begin(), perm.end(), 0);
    std::mt19937_64 rng(seed);
    const int64_t nb = n / bsz;  // whole batches only
    int64_t step = 0;
    std::vector<float> lh((size_t)std::min<int64_t>(nb, 4096));
    for (int ep = 0; ep < epochs && e == hipSuccess; ep++) {
        if (ep > 0) e = hipStreamSynchronize(s);  // the previous epoch's order has been uploaded
        if (e != hipSuccess) break;
        std::shuffle(perm.begin(), perm.end(), rng);
        e = hipMemcpyAsync(perm_d, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
        const float lr = epochs > 1 ? lr0 * std::pow(lr1 / lr0, (float)ep / (float)(epochs - 1)) : lr0;
        for (int64_t b = 0; b < nb && e == hipSuccess; b++) {
            e = mlp::gather_rows(x, 3, perm_d + b * bsz, bsz, xb, s);
            if (e == hipSuccess) e = mlp::gather_rows(y, kOut, perm_d + b * bsz, bsz, yb, s);
            if (e == hipSuccess) e = loss_grad_impl(params, xb, yb, !fp32_math, grad, lossd + (b % 4096), w, s);
            if (e == hipSuccess) e = mlp::adam(params, grad, m1, m2, kNParams, ++step, lr, s);
        }
        if (e == hipSuccess && loss_history) {
            const int64_t k = std::min<int64_t>(nb, 4096);
            e = hipMemcpyAsync(lh.data(), lossd, sizeof(float) * k, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            double sum = 0.0;
            for (int64_t i = 0; i < k; i++) sum += lh[i];
            loss_history[ep] = (float)(sum / (double)k);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (void *p : allocs) (void)hipFree(p);
    CK(e);
    return MATVIS_OK;
}

}  // extern "C"
