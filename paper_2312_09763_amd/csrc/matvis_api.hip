// Host side of libmatvis: the C ABI of include/matvis.h.
//
// A context owns every device buffer the hot path needs, sized once in
// matvis_init from the capacities in matvis_config, so matvis_simulate
// allocates nothing.  A simulate call walks (time batch) x (frequency batch)
// x (source chunk) and enqueues, per step of Alg. 2:
//   sky     : rotation + ordered horizon compaction of the chunk, per time;
//   interp  : beam at the visible sources, per (t, f) instance;
//   zform   : Z of Eq. (littlez), per instance;
//   herk    : V partials of Eq. (zz) over a device-built work list;
//   reduce  : fixed-order sum over k-splits and chunks, Hermitian fill.
// Nothing in the sequence waits on the host, so the whole call is captured
// once into a hipGraph (keyed by its arguments) and replayed afterwards.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "matvis.h"
#include "internal.h"
#include "mlp.h"

using namespace mv;

namespace {

struct GraphKey {
    std::vector<uint64_t> v;
    bool operator<(const GraphKey &o) const { return v < o.v; }
};

}  // namespace

struct matvis_ctx {
    matvis_config cfg{};
    int device = 0;
    int n_cu = 256;
    std::string err;
    hipStream_t last_stream = nullptr;
    hipStream_t capture_stream = nullptr;

    // derived geometry
    int N = 0, Np = 0, st = 128;
    int64_t chunk = 0, ldz = 0, ksplit = 4096;
    int max_splits = 1, ntb = 1, nfb = 1, herk_grid = 512, fused_grid = 256;
    int64_t nblk_cap = 1;
    bool fused = false;  // Z formed inside the product (FP32 / BF16X3)

    // device scratch
    double *xeq = nullptr, *rot = nullptr, *antc = nullptr, *s_hat = nullptr, *za_az = nullptr, *vacc = nullptr;
    double *xeq_in = nullptr;      // Eq. (xeq) in input order (before the sky-cell sort)
    int16_t *cell = nullptr;       // sky cell of each source
    int32_t *cell_hist = nullptr;  // per-block cell counts, then positions
    int32_t *perm = nullptr;       // source number at each sorted position
    int32_t *bidx = nullptr, *flags = nullptr, *blk_count = nullptr, *blk_off = nullptr, *count = nullptr,
            *idx = nullptr, *work = nullptr;
    void *A = nullptr, *Z = nullptr, *Z_lo = nullptr, *part = nullptr;
    std::vector<void *> allocs;

    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<GraphKey> graph_order;

    // per-step timing (matvis_profile_*)
    struct ProfRec {
        int kind;
        hipEvent_t a, b;
    };
    bool profiling = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> event_pool;

    // learned beam (beam_mode MATVIS_BEAM_SURROGATE)
    float *sur_P = nullptr;     // FP32 parameters, one network per unique beam
    __bf16 *sur_Wb = nullptr;   // bf16 W1..W4 LDS images, one per beam
    void *gridT = nullptr;      // channel-interleaved beam grids (grid beam modes, n_za >= 4)
    void *stencil = nullptr;    // per (slot, source) beam stencils of the batch (with gridT)
    double sur_nu0 = 0, sur_nu1 = 1;
    bool sur_set = false;

    // redundancy-aware sub-matrix product (matvis_set_pairs)
    bool pr_set = false;
    int32_t pr_n = 0, pr_tiles = 0;
    int64_t pr_size = 0;
    int32_t *pr_rows = nullptr;  // [tiles][2][ST] Z rows
    int32_t *pr_loc = nullptr;   // [n_pair][nf][nf][2]
    void *pr_part = nullptr;     // [B_cap][max_splits][tiles][ST][ST]
    void *pr_Z = nullptr, *pr_Z_lo = nullptr;  // fused contexts: Z of a batch for the pairs, when it fits
    double *pr_vacc = nullptr;   // [B_cap][n_pair][nf][nf] complex128
};

namespace {

matvis_status fail(matvis_ctx *c, matvis_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

matvis_status hip_fail(matvis_ctx *c, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, MATVIS_EHIP, m);
}

#define HIPCHK(ctx, expr)                                  \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

hipError_t take_event(matvis_ctx *c, hipEvent_t *e) {
    if (!c->event_pool.empty()) {
        *e = c->event_pool.back();
        c->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Launch `expr` (a hipError_t-returning launch helper) as part of step `kind`,
// bracketed by events when profiling.
#define STEP(ctx, kind, s, expr)                                        \
    do {                                                                \
        hipEvent_t _a = nullptr, _b = nullptr;                          \
        if ((ctx)->profiling) {                                         \
            HIPCHK(ctx, take_event(ctx, &_a));                          \
            HIPCHK(ctx, hipEventRecord(_a, s));                         \
        }                                                               \
        HIPCHK(ctx, expr);                                              \
        if ((ctx)->profiling) {                                         \
            HIPCHK(ctx, take_event(ctx, &_b));                          \
            HIPCHK(ctx, hipEventRecord(_b, s));                         \
            (ctx)->prof.push_back({(kind), _a, _b});                    \
        }                                                               \
    } while (0)

template <typename T>
matvis_status dalloc(matvis_ctx *c, T **p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, MATVIS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    c->allocs.push_back(q);
    *p = (T *)q;
    return MATVIS_OK;
}

int64_t round_up(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

size_t cbytes(int prec) { return prec == P64 ? 16 : 8; }  // bytes per complex of beams / Z / output

}  // namespace

// The library's k-split (Z columns per product work item) for a precision and
// product path when the configuration leaves it at 0.
int64_t mv::default_ksplit(int prec, bool over_sources, bool three_blocks) {
    return prec == P64                   ? 8192
           : prec == P32 && over_sources ? 8192
           : prec == P32                 ? 2048
           : over_sources                ? 20480
           : three_blocks                ? 8192
                                         : 4096;
}

namespace {

matvis_status validate_cfg(const matvis_config *c, std::string &why) {
    if (!c) return why = "config is NULL", MATVIS_EINVAL;
    if (c->n_ant <= 0) return why = "n_ant must be positive", MATVIS_EINVAL;
    if (c->n_feed != 1 && c->n_feed != 2) return why = "n_feed must be 1 or 2", MATVIS_EINVAL;
    if (c->n_ax != 1 && c->n_ax != 2) return why = "n_ax must be 1 or 2", MATVIS_EINVAL;
    if ((c->flags & MATVIS_FLAG_POLARISED_SKY) && c->n_ax != 2)
        return why = "a polarised sky needs the beam's two E-field axes (n_ax = 2)", MATVIS_EINVAL;
    if (c->n_beam <= 0) return why = "n_beam must be positive", MATVIS_EINVAL;
    if (c->max_src <= 0 || c->max_src > (int64_t)1 << 31) return why = "max_src out of range", MATVIS_EINVAL;
    if (c->max_time <= 0 || c->max_freq <= 0) return why = "max_time and max_freq must be positive", MATVIS_EINVAL;
    if (c->precision < MATVIS_FP64 || c->precision > MATVIS_BF16X3) return why = "unknown precision", MATVIS_EINVAL;
    if (c->beam_mode < MATVIS_BEAM_BILINEAR || c->beam_mode > MATVIS_BEAM_SURROGATE)
        return why = "unknown beam mode", MATVIS_EINVAL;
    if (c->beam_mode == MATVIS_BEAM_SURROGATE) {
        if (c->precision == MATVIS_FP64)
            return why = "the learned beam runs with FP32 or BF16X3 products", MATVIS_EUNSUPPORTED;
    } else {
        if (c->n_za < 3 || c->n_az < 3) return why = "beam grid must be at least 3 x 3", MATVIS_EINVAL;
        if (c->n_za >= 32768 || c->n_az >= 32768) return why = "beam grid must be below 32768 x 32768", MATVIS_EINVAL;
        if (!(c->dza_rad > 0) || !(c->daz_rad > 0)) return why = "grid spacings must be positive", MATVIS_EINVAL;
        if (std::fabs((c->n_za - 1) * c->dza_rad - M_PI / 2) > 1e-9)
            return why = "(n_za - 1) * dza_rad must equal pi/2 (za rows 0..90 deg)", MATVIS_EINVAL;
        if (std::fabs(c->n_az * c->daz_rad - 2 * M_PI) > 1e-9)
            return why = "n_az * daz_rad must equal 2 pi (periodic az)", MATVIS_EINVAL;
    }
    if (!std::isfinite(c->latitude_rad) || std::fabs(c->latitude_rad) > M_PI / 2)
        return why = "latitude out of range", MATVIS_EINVAL;
    if (c->src_chunk < 0 || c->batch_time < 0 || c->batch_freq < 0) return why = "negative batch sizes", MATVIS_EINVAL;
    if ((int64_t)c->n_ant * c->n_feed > 8192) return why = "n_ant * n_feed above 8192", MATVIS_EUNSUPPORTED;
    if (c->tile < 0 || (c->tile & ~0x5f) != 0 || ((c->tile & 15) != 0 && ((c->tile & 15) < 2 || (c->tile & 15) > 4)))
        return why = "tile: bits 0-3 (forming split) must be 0, 2, 3 or 4, bit 4 (block-pair kernel) and bit 6 "
                     "(stage depth) 0 or 1, no other bits", MATVIS_EINVAL;
    if (c->ksplit < 0 || c->ksplit % 64 != 0 || c->ksplit > ((int64_t)1 << 30))
        return why = "ksplit must be 0 or a positive multiple of 64", MATVIS_EINVAL;
    return MATVIS_OK;
}

}  // namespace

extern "C" {

const char *matvis_status_string(int32_t s) {
    switch (s) {
        case MATVIS_OK: return "MATVIS_OK";
        case MATVIS_EINVAL: return "MATVIS_EINVAL";
        case MATVIS_ENOMEM: return "MATVIS_ENOMEM";
        case MATVIS_EHIP: return "MATVIS_EHIP";
        case MATVIS_EUNSUPPORTED: return "MATVIS_EUNSUPPORTED";
        case MATVIS_ESTATE: return "MATVIS_ESTATE";
        case MATVIS_EDATA: return "MATVIS_EDATA";
        default: return "unknown status";
    }
}

void matvis_destroy(matvis_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &r : c->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    for (void *p : c->allocs) (void)hipFree(p);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
}

matvis_status matvis_init(const matvis_config *cfg, matvis_ctx **out) {
    if (!out) return MATVIS_EINVAL;
    *out = nullptr;
    std::string why;
    matvis_status st = validate_cfg(cfg, why);
    if (st != MATVIS_OK) {
        fprintf(stderr, "matvis_init: %s\n", why.c_str());
        return st;
    }
    matvis_ctx *c = new matvis_ctx();
    c->cfg = *cfg;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MATVIS_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    const int prec = cfg->precision;
    c->N = cfg->n_ant * cfg->n_feed;
    c->st = herk_super_tile(prec);
    c->Np = (int)round_up(c->N, c->st);
    // Sources per chunk.  Where Z goes through device memory its size sets the
    // chunk (2^18 sources); where the product forms Z itself only the per-source
    // buffers and the k-split partials grow with the chunk, so whole skies of up
    // to 2^22 sources go in one chunk: every chunk costs a launch of each step,
    // the load imbalance at the end of each product launch and a pass of the
    // reduction (on the 3.1M-pixel polarised sky one chunk instead of twelve was
    // 79.5 -> 71.7 ms per call of 8 instances).
    c->fused = prec != P64 && !(cfg->flags & MATVIS_FLAG_UNFUSED);
    c->chunk = cfg->src_chunk > 0 ? std::min<int64_t>(cfg->src_chunk, cfg->max_src)
                                  : std::min<int64_t>(cfg->max_src, (int64_t)1 << (c->fused ? 22 : 18));
    c->ldz = round_up((int64_t)cfg->n_ax * c->chunk, kColPad);
    // Columns per work item.  FP32 accumulators see ksplit / 2 sequential MFMA
    // updates per item; 2048 keeps that rounding near 2e-6 of the Cauchy-Schwarz
    // scale, and the items' partials are then summed in FP64.
    // Default k-split per precision: measured on the 128-antenna polarised workload,
    // err_CS grows about as sqrt(ksplit) (FP32: 3.1e-6 at 2048, 1.4e-5 at 8192;
    // BF16X3: 2.5e-6 at 4096, whose split error dominates below that).
    // The product over sources (two axes summed per source) accumulates ksplit / 2
    // sources per item: err_CS 3.5e-6 at 8192, 4.9e-6 at 16384, 7.0e-6 at 32768 on
    // the same workload; 20480 (~5.4e-6) keeps a factor 1.8 to 1e-5, and at the
    // benchmark's ~50 000 visible columns it gives three splits per instance
    // instead of four (fewer items and partials: 1.4 % of its step).
    const bool over_sources =
        c->fused && fused_path(prec, cfg->n_feed, cfg->n_ax, cfg->n_beam, cfg->n_ant, c->Np) == MATVIS_PATH_SOURCES;
    if (over_sources) c->Np = (int)round_up(c->N, 2 * c->st);  // whole blocks of 128 antennas x 2 feeds
    // FP32 product over sources: 8192 (err_CS 2.9e-6 on the benchmark instance,
    // against 0.8e-6 at 2048 and 1.5e-6 at 4096; the step 28.7 -> 27.3 ms).
    // scalar rows in three blocks (BF16X3): 8192 columns per split (err_CS 3.5e-6
    // against 2.8e-6 at 4096 on the 350-antenna diffuse sky, with half the partials:
    // its reduction went from 0.82 to 0.46 ms per two instances)
    const bool three_blocks =
        c->fused && fused_path(prec, cfg->n_feed, cfg->n_ax, cfg->n_beam, cfg->n_ant, c->Np) == MATVIS_PATH_FUSED_BLOCKS;
    c->ksplit = cfg->ksplit > 0 ? cfg->ksplit : default_ksplit(prec, over_sources, three_blocks);
    c->max_splits = (int)((c->ldz + c->ksplit - 1) / c->ksplit);
    // batch: all channels of a few times, enough instances to fill the GPU with
    // work items while keeping Z within a fixed share of device memory
    c->nfb = cfg->batch_freq > 0 ? std::min(cfg->batch_freq, cfg->max_freq) : std::min(cfg->max_freq, 16);
    // per-instance scratch that scales with the batch: Z (unfused only) and the k-split partials
    size_t zinst = (c->fused ? 0 : (size_t)c->Np * c->ldz * cbytes(prec)) +
                   (size_t)c->max_splits * c->Np * c->Np * cbytes(prec);
    size_t budget = (size_t)12 << 30;
    int ntb_auto = (int)std::max<size_t>(1, budget / std::max<size_t>(1, zinst * c->nfb));
    c->ntb = cfg->batch_time > 0 ? cfg->batch_time : std::min(ntb_auto, 16);
    c->ntb = std::max(1, std::min(c->ntb, cfg->max_time));
    const int B = c->ntb * c->nfb;
    c->nblk_cap = std::max<int64_t>((c->chunk + 255) / 256, 1);
    int64_t nblk_total = std::max<int64_t>(c->nblk_cap * c->ntb, (cfg->max_src + 255) / 256);
    int occ = std::max(1, herk_occupancy(prec));
    c->herk_grid = std::max(8, (c->n_cu * occ / 8) * 8);
    if (c->fused) c->fused_grid = std::max(8, (c->n_cu * std::max(1, herk_fused_occupancy(prec)) / 8) * 8);
    // Z scratch: a whole batch when Z goes through device memory, else one
    // instance (used only by matvis_step_herk)
    const int zinst_n = c->fused ? 1 : B;

    const size_t ncomp = (size_t)cfg->n_beam * cfg->n_feed * cfg->n_ax;
#define ALLOC(ptr, bytes)                              \
    do {                                               \
        matvis_status _s = dalloc(c, &(ptr), (bytes)); \
        if (_s != MATVIS_OK) {                         \
            fprintf(stderr, "matvis_init: %s\n", c->err.c_str()); \
            matvis_destroy(c);                         \
            return _s;                                 \
        }                                              \
    } while (0)
    ALLOC(c->xeq, sizeof(double) * 3 * cfg->max_src);
    ALLOC(c->xeq_in, sizeof(double) * 3 * cfg->max_src);
    ALLOC(c->cell, sizeof(int16_t) * cfg->max_src);
    ALLOC(c->cell_hist, sizeof(int32_t) * sort_hist_entries(cfg->max_src));
    ALLOC(c->perm, sizeof(int32_t) * cfg->max_src);
    ALLOC(c->rot, sizeof(double) * 9 * cfg->max_time);
    ALLOC(c->antc, sizeof(double) * 3 * cfg->n_ant);
    ALLOC(c->bidx, sizeof(int32_t) * cfg->n_ant);
    ALLOC(c->flags, sizeof(int32_t) * 4);
    ALLOC(c->blk_count, sizeof(int32_t) * nblk_total);
    ALLOC(c->blk_off, sizeof(int32_t) * nblk_total);
    ALLOC(c->count, sizeof(int32_t) * std::max(c->ntb, 1));
    ALLOC(c->idx, sizeof(int32_t) * c->ntb * c->chunk);
    ALLOC(c->s_hat, sizeof(double) * 3 * c->ntb * c->chunk);
    ALLOC(c->za_az, sizeof(double) * 2 * c->ntb * c->chunk);
    ALLOC(c->A, cbytes(prec) * ncomp * B * c->chunk);
    const size_t zbytes = (prec == PB3 ? (size_t)4 : cbytes(prec)) * zinst_n * c->Np * c->ldz;
    ALLOC(c->Z, zbytes);
    if (prec == PB3) ALLOC(c->Z_lo, zbytes);
    ALLOC(c->part, cbytes(prec) * B * (size_t)c->max_splits * c->Np * c->Np);
    if (c->chunk < cfg->max_src) ALLOC(c->vacc, sizeof(double) * 2 * B * (size_t)c->N * c->N);
    ALLOC(c->work, sizeof(int32_t) * (3 * B + 1));  // item prefix, then k-splits and columns per split
    if (cfg->beam_mode != MATVIS_BEAM_SURROGATE && cfg->n_za >= 4) {
        ALLOC(c->gridT, cbytes(prec) * (size_t)grid_interleave_elems(cfg->n_beam, cfg->max_freq,
                                                                     cfg->n_feed * cfg->n_ax, cfg->n_za, cfg->n_az));
        ALLOC(c->stencil, interp_stencil_bytes(prec, c->chunk, c->ntb));
    }
    if (cfg->beam_mode == MATVIS_BEAM_SURROGATE) {
        ALLOC(c->sur_P, sizeof(float) * kNParams * cfg->n_beam);
        ALLOC(c->sur_Wb, sizeof(__bf16) * mlp::kImgElems * cfg->n_beam);
    }
#undef ALLOC
    // Rows N..Np-1 of Z are never written by the kernels and must read as zero.
    hipError_t e = hipMemset(c->Z, 0, zbytes);
    if (e == hipSuccess && c->Z_lo) e = hipMemset(c->Z_lo, 0, zbytes);
    if (e == hipSuccess) e = hipMemset(c->flags, 0, sizeof(int32_t) * 4);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        fprintf(stderr, "matvis_init: %s\n", hipGetErrorString(e));
        matvis_destroy(c);
        return MATVIS_EHIP;
    }
    *out = c;
    return MATVIS_OK;
}

const char *matvis_last_error(const matvis_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

matvis_status matvis_finish(matvis_ctx *c) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->last_stream));
    int32_t h[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpy(h, c->flags, sizeof(h), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemset(c->flags, 0, sizeof(h)));
    HIPCHK(c, hipDeviceSynchronize());
    if (h[0]) {
        std::string m = "invalid input data:";
        if (h[0] & FLAG_BAD_FLUX) m += " negative or non-finite flux;";
        if (h[0] & FLAG_BAD_ANTPOS) m += " non-finite antenna position;";
        if (h[0] & FLAG_BAD_BEAM_IDX) m += " beam index out of range;";
        return fail(c, MATVIS_EDATA, m);
    }
    return MATVIS_OK;
}

}  // extern "C"

namespace {

// Enqueue the whole simulate sequence on stream s (no host waits).
matvis_status enqueue_simulate(matvis_ctx *c, const double *antpos, const int32_t *beam_idx, const double *freqs,
                               int32_t n_freq, const double *lsts, int32_t n_time, const double *radec, int64_t n_src,
                               const double *flux, const void *grid, void *vis, hipStream_t s, bool pairs = false) {
    const matvis_config &g = c->cfg;
    const int prec = g.precision;
    const int pol = (g.flags & MATVIS_FLAG_POLARISED_SKY) ? 1 : 0;
    STEP(c, MATVIS_STEP_OTHER, s,
         launch_prep_inputs(antpos, g.n_ant, beam_idx, g.n_beam, flux, (int64_t)n_freq * n_src, pol, c->antc,
                            c->bidx, c->flags, s));
    STEP(c, MATVIS_STEP_SKY, s,
         launch_xeq_sorted(radec, n_src, g.max_src, SortBufs{c->xeq_in, c->cell, c->cell_hist, c->perm}, c->xeq, s));
    if (c->gridT)
        STEP(c, MATVIS_STEP_BEAM, s,
             launch_grid_interleave(prec, grid, g.n_beam, n_freq, g.n_feed * g.n_ax, g.n_za, g.n_az, c->gridT, s));
    STEP(c, MATVIS_STEP_SKY, s, launch_rotmats(lsts, n_time, g.latitude_rad, c->rot, s));
    const int64_t n_chunks = std::max<int64_t>(1, (n_src + c->chunk - 1) / c->chunk);
    const int ncomp = g.n_feed * g.n_ax;
    const int B_cap = c->ntb * c->nfb;  // instances the batch buffers hold
    for (int t0 = 0; t0 < n_time; t0 += c->ntb) {
        const int ntb = std::min(c->ntb, n_time - t0);
        for (int f0 = 0; f0 < n_freq; f0 += c->nfb) {
            const int nfb = std::min(c->nfb, n_freq - f0);
            Batch bt{t0, f0, ntb, nfb, ntb * nfb};
            for (int64_t ch = 0; ch < n_chunks; ch++) {
                const int64_t c0 = ch * c->chunk;
                const int64_t ns = std::min(c->chunk, n_src - c0);
                SkyBufs sb{c->xeq,   g.max_src, c->rot,   c->blk_count, c->blk_off, c->count,
                           c->idx,   c->s_hat,  c->za_az, c->chunk,     c->perm};
                if (n_chunks > 1 || f0 == 0) STEP(c, MATVIS_STEP_SKY, s, launch_sky(sb, t0, ntb, c0, ns, s));

                InterpArgs ia{};
                ia.grid = c->gridT ? c->gridT : grid;
                ia.n_freq_grid = n_freq;
                ia.n_beam = g.n_beam;
                ia.n_feed = g.n_feed;
                ia.n_ax = g.n_ax;
                ia.n_za = g.n_za;
                ia.n_az = g.n_az;
                ia.dza = g.dza_rad;
                ia.daz = g.daz_rad;
                ia.za_az = c->za_az;
                ia.stencil = c->stencil;
                ia.count = c->count;
                ia.ld_src = c->chunk;
                ia.A = c->A;
                ia.max_m = ns;
                // The beam step carries the sky into B (sqrt(I) A, or A M for a polarised sky)
                // whenever the product forms Z itself, and always for a polarised sky.
                if (c->fused || pol) {
                    ia.idx = c->idx;
                    ia.flux = flux;
                    ia.n_src = n_src;
                    ia.pol = pol;
                    ia.stokes_stride = (int64_t)n_freq * n_src;
                }
                if (g.beam_mode == MATVIS_BEAM_SURROGATE)
                    for (int b = 0; b < g.n_beam; b++)  // one network per unique beam
                        STEP(c, MATVIS_STEP_BEAM, s,
                             mlp::infer_sim(c->sur_P + (size_t)b * kNParams, c->sur_Wb + (size_t)b * mlp::kImgElems,
                                            c->sur_nu0, c->sur_nu1, c->za_az, c->count, ia.idx, flux, n_src, pol,
                                            ia.stokes_stride, freqs, c->chunk, ns, c->A, g.n_feed, g.n_ax, b,
                                            g.n_beam, bt, s));
                else
                    STEP(c, MATVIS_STEP_BEAM, s,
                         c->gridT ? launch_interp_tf(prec, g.beam_mode, ia, bt, s)
                                  : launch_interp(prec, g.beam_mode, ia, bt, s));

                HerkArgs ha{};
                ha.Z = c->Z;
                ha.Z_lo = c->Z_lo;
                ha.ldz = c->ldz;
                ha.inst_stride = (int64_t)c->Np * c->ldz;
                ha.n_rows = c->N;
                ha.n_rows_pad = c->Np;
                ha.count = c->count;
                ha.n_ax = g.n_ax;
                ha.nfb = nfb;
                ha.n_inst = bt.n_inst;
                ha.ksplit = c->ksplit;
                ha.max_splits = c->max_splits;
                ha.part = c->part;
                ha.work = c->work;
                ha.nsplit = c->work + B_cap + 1;
                ha.kcols = c->work + 2 * B_cap + 1;
                ha.balance_grid = c->fused ? c->fused_grid : 0;
                ha.grid = c->herk_grid;
                if (!pairs) STEP(c, MATVIS_STEP_OTHER, s, launch_worklist(prec, ha, c->fused ? 1 : 0, s));

                if (c->fused && !pairs) {
                    FusedArgs fa{};
                    fa.antc = c->antc;
                    fa.bidx = c->bidx;
                    fa.freqs = freqs;
                    fa.s_hat = c->s_hat;
                    fa.B = c->A;
                    fa.count = c->count;
                    fa.ld_src = c->chunk;
                    fa.n_ant = g.n_ant;
                    fa.n_feed = g.n_feed;
                    fa.n_ax = g.n_ax;
                    fa.n_beam = g.n_beam;
                    fa.n_rows_pad = c->Np;
                    fa.f0 = f0;
                    fa.nfb = nfb;
                    fa.n_inst = bt.n_inst;
                    fa.kcols = ha.kcols;
                    fa.max_splits = c->max_splits;
                    fa.part = c->part;
                    fa.work = c->work;
                    fa.grid = c->fused_grid;
                    fa.tile = g.tile;
                    if (c->profiling && fused_has_pairs(prec, fa)) {  // time the two launches apart
                        STEP(c, MATVIS_STEP_HERK, s, launch_herk_fused(prec, fa, s, FUSED_FIRST));
                        STEP(c, MATVIS_STEP_HERK_PAIRS, s, launch_herk_fused(prec, fa, s, FUSED_PAIRS));
                    } else {
                        STEP(c, MATVIS_STEP_HERK, s, launch_herk_fused(prec, fa, s));
                    }
                }

                ZformArgs za{};
                za.antc = c->antc;
                za.bidx = c->bidx;
                za.freqs = freqs;
                za.flux = pol ? nullptr : flux;  // a polarised sky is already in A
                za.n_src = n_src;
                za.idx = c->idx;
                za.s_hat = c->s_hat;
                za.count = c->count;
                za.A = c->A;
                za.ld_src = c->chunk;
                za.n_ant = g.n_ant;
                za.n_feed = g.n_feed;
                za.n_ax = g.n_ax;
                za.n_beam = g.n_beam;
                za.Z = c->Z;
                za.Z_lo = c->Z_lo;
                za.ldz = c->ldz;
                za.n_rows_pad = c->Np;
                za.max_m = (round_up(g.n_ax * ns, kColPad) + g.n_ax - 1) / g.n_ax;
                if (!c->fused) {
                    STEP(c, MATVIS_STEP_ZFORM, s, launch_zform(prec, za, bt, s));
                    if (!pairs) STEP(c, MATVIS_STEP_HERK, s, launch_herk(prec, ha, s));
                } else if (pairs && c->pr_Z) {
                    // the pairs of a fused context with room for a batch of Z: form Z once
                    // (B already carries the sky) rather than once per sub-matrix tile
                    za.flux = nullptr;
                    za.Z = c->pr_Z;
                    za.Z_lo = c->pr_Z_lo;
                    STEP(c, MATVIS_STEP_ZFORM, s, launch_zform(prec, za, bt, s));
                }
                if (pairs) {
                    // App. A: only the planned sub-matrices, then the requested pairs
                    SubmatArgs sa{};
                    sa.Z = c->fused ? c->pr_Z : c->Z;
                    sa.Z_lo = c->fused ? c->pr_Z_lo : c->Z_lo;
                    sa.ldz = c->ldz;
                    sa.inst_stride = (int64_t)c->Np * c->ldz;
                    sa.rows = c->pr_rows;
                    sa.n_tiles = c->pr_tiles;
                    sa.count = c->count;
                    sa.n_ax = g.n_ax;
                    sa.nfb = nfb;
                    sa.n_inst = bt.n_inst;
                    sa.ksplit = c->ksplit;
                    sa.max_splits = c->max_splits;
                    sa.part = c->pr_part;
                    if (c->fused && !c->pr_Z) {  // Z formed in the stages from B = sqrt(I) A and the fringe phase
                        sa.antc = c->antc;
                        sa.bidx = c->bidx;
                        sa.freqs = freqs;
                        sa.s_hat = c->s_hat;
                        sa.B = c->A;
                        sa.ld_src = c->chunk;
                        sa.n_feed = g.n_feed;
                        sa.n_beam = g.n_beam;
                        sa.f0 = f0;
                        STEP(c, MATVIS_STEP_HERK, s, launch_submat_fused(prec, sa, s));
                    } else {
                        STEP(c, MATVIS_STEP_HERK, s, launch_submat(prec, sa, s));
                    }
                    SubmatReduceArgs sr{};
                    sr.part = c->pr_part;
                    sr.n_tiles = c->pr_tiles;
                    sr.max_splits = c->max_splits;
                    sr.st = kSubmatTile;
                    sr.loc = c->pr_loc;
                    sr.n_pair = c->pr_n;
                    sr.n_feed = g.n_feed;
                    sr.count = c->count;
                    sr.n_ax = g.n_ax;
                    sr.nfb = nfb;
                    sr.n_inst = bt.n_inst;
                    sr.ksplit = c->ksplit;
                    sr.vacc = c->pr_vacc;
                    sr.first = ch == 0;
                    sr.last = ch == n_chunks - 1;
                    sr.out = vis;
                    sr.n_freq_total = n_freq;
                    sr.bt = bt;
                    STEP(c, MATVIS_STEP_REDUCE, s, launch_submat_reduce(prec, sr, s));
                    continue;
                }

                ReduceArgs ra{};
                ra.part = c->part;
                ra.n_rows = c->N;
                ra.n_rows_pad = c->Np;
                ra.max_splits = c->max_splits;
                ra.count = c->count;
                ra.n_ax = g.n_ax;
                ra.nfb = nfb;
                ra.n_inst = bt.n_inst;
                ra.ksplit = c->ksplit;
                ra.nsplit = ha.nsplit;
                ra.vacc = c->vacc;
                ra.first = ch == 0;
                ra.last = ch == n_chunks - 1;
                ra.out = vis;
                ra.out_kind = 0;
                ra.n_ant = g.n_ant;
                ra.n_feed = g.n_feed;
                ra.n_freq_total = n_freq;
                ra.bt = bt;
                STEP(c, MATVIS_STEP_REDUCE, s, launch_reduce(prec, ra, s));
            }
        }
    }
    (void)ncomp;
    return MATVIS_OK;
}

matvis_status simulate_impl(matvis_ctx *c, const double *antpos, const int32_t *beam_idx, const double *freqs,
                            int32_t n_freq, const double *lsts, int32_t n_time, const double *src_radec,
                            int64_t n_src, const double *src_flux, const void *beam_grid, void *vis, void *stream,
                            bool pairs) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    const matvis_config &g = c->cfg;
    if (!antpos || !freqs || !lsts || !vis) return fail(c, MATVIS_EINVAL, "a required pointer is NULL");
    if (n_src > 0 && (!src_radec || !src_flux)) return fail(c, MATVIS_EINVAL, "src_radec or src_flux is NULL");
    if (g.beam_mode == MATVIS_BEAM_SURROGATE) {
        if (!c->sur_set) return fail(c, MATVIS_ESTATE, "no learned beam loaded (call matvis_set_surrogate)");
    } else if (!beam_grid) {
        return fail(c, MATVIS_EINVAL, "beam_grid is NULL");
    }
    if (n_freq <= 0 || n_freq > g.max_freq) return fail(c, MATVIS_EINVAL, "n_freq outside [1, max_freq]");
    if (n_time <= 0 || n_time > g.max_time) return fail(c, MATVIS_EINVAL, "n_time outside [1, max_time]");
    if (n_src < 0 || n_src > g.max_src) return fail(c, MATVIS_EINVAL, "n_src outside [0, max_src]");
    if (c->chunk < g.max_src && !c->vacc) return fail(c, MATVIS_ESTATE, "chunk accumulator missing");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    c->last_stream = s;
    if (n_src == 0) {
        const size_t per = pairs ? (size_t)c->pr_n : (size_t)g.n_ant * g.n_ant;
        const size_t vb = cbytes(g.precision) * (size_t)n_time * n_freq * per * g.n_feed * g.n_feed;
        HIPCHK(c, hipMemsetAsync(vis, 0, vb, s));
        return MATVIS_OK;
    }
    if ((g.flags & MATVIS_FLAG_NO_GRAPH) || c->profiling)
        return enqueue_simulate(c, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux, beam_grid,
                                vis, s, pairs);
    GraphKey key;
    key.v = {(uint64_t)antpos, (uint64_t)beam_idx, (uint64_t)freqs, (uint64_t)n_freq, (uint64_t)lsts,
             (uint64_t)n_time, (uint64_t)src_radec, (uint64_t)n_src, (uint64_t)src_flux, (uint64_t)beam_grid,
             (uint64_t)vis, (uint64_t)pairs};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
        matvis_status st = enqueue_simulate(c, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src,
                                            src_flux, beam_grid, vis, c->capture_stream, pairs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
        if (st != MATVIS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        if (c->graph_order.size() >= 8) {
            auto old = c->graphs.find(c->graph_order.front());
            if (old != c->graphs.end()) {
                (void)hipGraphExecDestroy(old->second);
                c->graphs.erase(old);
            }
            c->graph_order.erase(c->graph_order.begin());
        }
        it = c->graphs.emplace(key, exec).first;
        c->graph_order.push_back(key);
    }
    HIPCHK(c, hipGraphLaunch(it->second, s));
    return MATVIS_OK;
}

}  // namespace

extern "C" {

matvis_status matvis_simulate(matvis_ctx *c, const double *antpos, const int32_t *beam_idx, const double *freqs,
                              int32_t n_freq, const double *lsts, int32_t n_time, const double *src_radec,
                              int64_t n_src, const double *src_flux, const void *beam_grid, void *vis, void *stream) {
    return simulate_impl(c, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux, beam_grid,
                         vis, stream, false);
}

matvis_status matvis_simulate_pairs(matvis_ctx *c, const double *antpos, const int32_t *beam_idx,
                                    const double *freqs, int32_t n_freq, const double *lsts, int32_t n_time,
                                    const double *src_radec, int64_t n_src, const double *src_flux,
                                    const void *beam_grid, void *vis_pairs, void *stream) {
    if (!c) return MATVIS_EINVAL;
    if (!c->pr_set) return fail(c, MATVIS_ESTATE, "no pair plan (call matvis_set_pairs)");
    return simulate_impl(c, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux, beam_grid,
                         vis_pairs, stream, true);
}

matvis_status matvis_set_pairs(matvis_ctx *c, const int32_t *pair_a, const int32_t *pair_b, int32_t n_pair,
                               int32_t n_sub, int64_t *size_out) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    const matvis_config &g = c->cfg;
    if (!pair_a || !pair_b || n_pair <= 0 || n_sub <= 0) return fail(c, MATVIS_EINVAL, "need pairs and n_sub >= 1");
    for (int u = 0; u < n_pair; u++)
        if (pair_a[u] < 0 || pair_a[u] >= g.n_ant || pair_b[u] < 0 || pair_b[u] >= g.n_ant)
            return fail(c, MATVIS_EINVAL, "pair antenna outside [0, n_ant)");
    const red::Plan P = red::plan(pair_a, pair_b, n_pair, g.n_ant, n_sub);
    const int nf = g.n_feed, ST = kSubmatTile;
    // tiles of every sub-matrix over its Z rows (antenna a, feed p -> row a nf + p)
    std::vector<int32_t> rows, base;
    std::vector<int> ntc;
    int64_t size = 0;
    for (size_t x = 0; x < P.A.size(); x++) {
        const int ra = (int)P.A[x].size() * nf, rb = (int)P.B[x].size() * nf;
        const int nta = (ra + ST - 1) / ST, ntb = (rb + ST - 1) / ST;
        base.push_back((int32_t)(rows.size() / (2 * ST)));
        ntc.push_back(ntb);
        size += (int64_t)P.A[x].size() * P.B[x].size();
        for (int ti = 0; ti < nta; ti++)
            for (int tj = 0; tj < ntb; tj++) {
                for (int r = 0; r < ST; r++) {
                    const int q = ti * ST + r;
                    rows.push_back(q < ra ? P.A[x][q / nf] * nf + q % nf : -1);
                }
                for (int r = 0; r < ST; r++) {
                    const int q = tj * ST + r;
                    rows.push_back(q < rb ? P.B[x][q / nf] * nf + q % nf : -1);
                }
            }
    }
    const int n_tiles = (int)(rows.size() / (2 * ST));
    std::vector<int> sub_of(g.n_ant, -1), pos_in(g.n_ant, -1);
    for (size_t x = 0; x < P.A.size(); x++)
        for (size_t i = 0; i < P.A[x].size(); i++) {
            sub_of[P.A[x][i]] = (int)x;
            pos_in[P.A[x][i]] = (int)i;
        }
    std::vector<int32_t> loc((size_t)n_pair * nf * nf * 2);
    for (int u = 0; u < n_pair; u++) {
        const int x = sub_of[pair_a[u]];
        const auto &B = P.B[x];
        const int ib = (int)(std::lower_bound(B.begin(), B.end(), pair_b[u]) - B.begin());
        for (int p = 0; p < nf; p++)
            for (int q = 0; q < nf; q++) {
                const int r = pos_in[pair_a[u]] * nf + p, col = ib * nf + q;
                const size_t e = (((size_t)u * nf + p) * nf + q) * 2;
                loc[e] = base[x] + (r / ST) * ntc[x] + col / ST;
                loc[e + 1] = (r % ST) * ST + col % ST;
            }
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    // graphs captured with an earlier plan hold its buffers
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->graph_order.clear();
    for (void *q : {(void *)c->pr_rows, (void *)c->pr_loc, c->pr_part, (void *)c->pr_vacc, c->pr_Z, c->pr_Z_lo}) {
        if (!q) continue;
        auto it = std::find(c->allocs.begin(), c->allocs.end(), q);
        if (it != c->allocs.end()) c->allocs.erase(it);
        (void)hipFree(q);
    }
    c->pr_rows = c->pr_loc = nullptr;
    c->pr_part = nullptr;
    c->pr_vacc = nullptr;
    c->pr_Z = c->pr_Z_lo = nullptr;
    c->pr_set = false;
    const int B_cap = c->ntb * c->nfb;
    matvis_status st;
    if ((st = dalloc(c, &c->pr_rows, sizeof(int32_t) * rows.size())) != MATVIS_OK) return st;
    if ((st = dalloc(c, &c->pr_loc, sizeof(int32_t) * loc.size())) != MATVIS_OK) return st;
    if ((st = dalloc(c, &c->pr_part, cbytes(g.precision) * (size_t)B_cap * c->max_splits * n_tiles * ST * ST)) !=
        MATVIS_OK)
        return st;
    if ((st = dalloc(c, &c->pr_vacc, sizeof(double) * 2 * (size_t)B_cap * n_pair * nf * nf)) != MATVIS_OK) return st;
    // Fused contexts: a sub-matrix tile reuses a formed Z row only within its 32
    // rows, so forming Z once per batch in device memory is faster whenever it
    // fits a fixed budget; otherwise the tiles form their rows in the stages.
    if (c->fused) {
        const size_t zplane = (g.precision == PB3 ? (size_t)4 : cbytes(g.precision)) * B_cap * c->Np * c->ldz;
        if (zplane * (g.precision == PB3 ? 2 : 1) <= ((size_t)8 << 30)) {
            if ((st = dalloc(c, &c->pr_Z, zplane)) != MATVIS_OK) return st;
            if (g.precision == PB3 && (st = dalloc(c, &c->pr_Z_lo, zplane)) != MATVIS_OK) return st;
        }
    }
    HIPCHK(c, hipMemcpy(c->pr_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->pr_loc, loc.data(), sizeof(int32_t) * loc.size(), hipMemcpyHostToDevice));
    c->pr_n = n_pair;
    c->pr_tiles = n_tiles;
    c->pr_size = size;
    c->pr_set = true;
    if (size_out) *size_out = size;
    return MATVIS_OK;
}

matvis_status matvis_set_surrogate(matvis_ctx *c, const float *params, double nu_min_hz, double nu_max_hz) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    if (c->cfg.beam_mode != MATVIS_BEAM_SURROGATE)
        return fail(c, MATVIS_ESTATE, "context was not created with beam_mode MATVIS_BEAM_SURROGATE");
    if (!params) return fail(c, MATVIS_EINVAL, "params is NULL");
    if (!std::isfinite(nu_min_hz) || !std::isfinite(nu_max_hz) || !(nu_max_hz > nu_min_hz))
        return fail(c, MATVIS_EINVAL, "need finite nu_min_hz < nu_max_hz");
    HIPCHK(c, hipSetDevice(c->device));
    // kernels already captured hold the old normalisation by value
    HIPCHK(c, hipDeviceSynchronize());
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->graph_order.clear();
    HIPCHK(c, hipMemcpy(c->sur_P, params, sizeof(float) * kNParams * c->cfg.n_beam, hipMemcpyDeviceToDevice));
    for (int b = 0; b < c->cfg.n_beam; b++)
        HIPCHK(c, mlp::pack_weights(c->sur_P + (size_t)b * kNParams, c->sur_Wb + (size_t)b * mlp::kImgElems, nullptr));
    HIPCHK(c, hipDeviceSynchronize());
    c->sur_nu0 = nu_min_hz;
    c->sur_nu1 = nu_max_hz;
    c->sur_set = true;
    return MATVIS_OK;
}

int32_t matvis_product_path_of(const matvis_ctx *c) {
    if (!c) return MATVIS_EINVAL;
    if (!c->fused) return MATVIS_PATH_Z_IN_HBM;
    const matvis_config &g = c->cfg;
    return fused_path(g.precision == MATVIS_FP32 ? P32 : g.precision == MATVIS_BF16X3 ? PB3 : P64, g.n_feed, g.n_ax,
                      g.n_beam, g.n_ant, c->Np);
}

matvis_status matvis_profile_enable(matvis_ctx *c, int32_t enable) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    c->profiling = enable != 0;
    return MATVIS_OK;
}

matvis_status matvis_profile_read(matvis_ctx *c, double *ms, int64_t *launches) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    if (!ms || !launches) return fail(c, MATVIS_EINVAL, "output arrays are NULL");
    for (int k = 0; k < MATVIS_N_STEPS; k++) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    HIPCHK(c, hipSetDevice(c->device));
    matvis_status st = MATVIS_OK;
    for (auto &r : c->prof) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && st == MATVIS_OK) st = hip_fail(c, e, "hipEventElapsedTime");
        ms[r.kind] += t;
        launches[r.kind] += 1;
        c->event_pool.push_back(r.a);
        c->event_pool.push_back(r.b);
    }
    c->prof.clear();
    return st;
}

matvis_status matvis_step_sky(matvis_ctx *c, const double *lsts, int32_t n_time, const double *src_radec,
                              int64_t n_src, int32_t *idx, int32_t *count, double *s_hat, double *za_az,
                              void *stream) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    const matvis_config &g = c->cfg;
    if (!lsts || !src_radec || !idx || !count || !s_hat || !za_az)
        return fail(c, MATVIS_EINVAL, "a required pointer is NULL");
    if (n_time <= 0 || n_time > g.max_time) return fail(c, MATVIS_EINVAL, "n_time outside [1, max_time]");
    if (n_src <= 0 || n_src > g.max_src) return fail(c, MATVIS_EINVAL, "n_src outside [1, max_src]");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    c->last_stream = s;
    HIPCHK(c, launch_xeq(src_radec, n_src, c->xeq, g.max_src, s));
    HIPCHK(c, launch_rotmats(lsts, n_time, g.latitude_rad, c->rot, s));
    for (int t = 0; t < n_time; t++) {
        SkyBufs sb{c->xeq, g.max_src, c->rot, c->blk_count, c->blk_off, count + t, idx + (int64_t)t * n_src,
                   s_hat + (int64_t)t * 3 * n_src, za_az + (int64_t)t * 2 * n_src, n_src};
        HIPCHK(c, launch_sky(sb, t, 1, 0, n_src, s));
    }
    return MATVIS_OK;
}

matvis_status matvis_step_interp(matvis_ctx *c, const double *za_az, int64_t n, const void *grid, void *A,
                                 void *stream) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    const matvis_config &g = c->cfg;
    if (!za_az || !grid || !A) return fail(c, MATVIS_EINVAL, "a required pointer is NULL");
    if (n < 0) return fail(c, MATVIS_EINVAL, "n must be non-negative");
    if (g.beam_mode == MATVIS_BEAM_SURROGATE) return fail(c, MATVIS_EUNSUPPORTED, "grid interpolation not selected");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    c->last_stream = s;
    InterpArgs ia{};
    ia.grid = grid;
    ia.n_freq_grid = 1;
    ia.n_beam = g.n_beam;
    ia.n_feed = g.n_feed;
    ia.n_ax = g.n_ax;
    ia.n_za = g.n_za;
    ia.n_az = g.n_az;
    ia.dza = g.dza_rad;
    ia.daz = g.daz_rad;
    ia.za_az = za_az;
    ia.count = nullptr;
    ia.fixed_count = n;
    ia.ld_src = n;
    ia.A = A;
    ia.max_m = n;
    Batch bt{0, 0, 1, 1, 1};
    HIPCHK(c, launch_interp(g.precision, g.beam_mode, ia, bt, s));
    return MATVIS_OK;
}

matvis_status matvis_step_herk(matvis_ctx *c, const void *Zin, int32_t n_row, int64_t n_col, int64_t ld, void *V,
                               void *stream) {
    if (!c) return MATVIS_EINVAL;
    c->err.clear();
    const matvis_config &g = c->cfg;
    if (!Zin || !V) return fail(c, MATVIS_EINVAL, "a required pointer is NULL");
    if (n_row <= 0 || n_row > c->N) return fail(c, MATVIS_EINVAL, "n_row outside [1, n_ant * n_feed]");
    if (n_col < 0 || n_col > c->ldz) return fail(c, MATVIS_EINVAL, "n_col above the context's column capacity");
    if (ld < n_col) return fail(c, MATVIS_EINVAL, "ld smaller than n_col");
    const int prec = g.precision;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    c->last_stream = s;
    const int np = (int)round_up(n_row, c->st);
    const int64_t ncp = round_up(n_col, kColPad);
    HIPCHK(c, launch_z_import(prec, Zin, n_row, np, n_col, ld, c->Z, c->Z_lo, c->ldz, ncp, s));
    HerkArgs ha{};
    ha.Z = c->Z;
    ha.Z_lo = c->Z_lo;
    ha.ldz = c->ldz;
    ha.inst_stride = (int64_t)np * c->ldz;
    ha.n_rows = n_row;
    ha.n_rows_pad = np;
    ha.count = nullptr;
    ha.fixed_k = n_col;
    ha.n_ax = 1;
    ha.nfb = 1;
    ha.n_inst = 1;
    ha.ksplit = c->ksplit;
    ha.max_splits = c->max_splits;
    ha.part = c->part;
    ha.work = c->work;
    ha.nsplit = c->work + c->ntb * c->nfb + 1;
    ha.kcols = c->work + 2 * c->ntb * c->nfb + 1;
    ha.balance_grid = 0;
    ha.grid = c->herk_grid;
    HIPCHK(c, launch_worklist(prec, ha, 0, s));
    HIPCHK(c, launch_herk(prec, ha, s));
    ReduceArgs ra{};
    ra.part = c->part;
    ra.n_rows = n_row;
    ra.n_rows_pad = np;
    ra.max_splits = c->max_splits;
    ra.count = nullptr;
    ra.fixed_k = n_col;
    ra.n_ax = 1;
    ra.nfb = 1;
    ra.n_inst = 1;
    ra.ksplit = c->ksplit;
    ra.vacc = nullptr;
    ra.first = 1;
    ra.last = 1;
    ra.out = V;
    ra.out_kind = 1;
    ra.n_ant = g.n_ant;
    ra.n_feed = g.n_feed;
    ra.n_freq_total = 1;
    ra.bt = Batch{0, 0, 1, 1, 1};
    HIPCHK(c, launch_reduce(prec, ra, s));
    return MATVIS_OK;
}

}  // extern "C"
