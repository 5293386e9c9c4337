// Autotuner for the batched product (matvis_autotune in include/matvis.h).
//
// The knobs are discrete, so they are searched on the caller's own inputs by
// coordinate descent from the library's defaults: one axis at a time, every
// value of the axis is timed with the other axes at their best so far, and
// the axis keeps its fastest value.  The axes, in order:
//   pair kernel the kernel of the off-diagonal antenna-block pairs (product
//               over sources, BF16X3): one-sided or square-root weights;
//   tile        the forming split: rows per stage formed by the multiply-first
//               waves (paths that split the forming between two wave kinds);
//   stage       sources per stage, 32 or 16 (BF16X3 three-block path);
//   ksplit      Z columns per work item: the path's default, two and four times it
//               (fewer partial sums; each FP32 accumulator sees more terms, so
//               its rounding grows about as the square root of the split), and
//               its halves and quarters (more accurate than the default);
//   src_chunk   sources per chunk: the default and 2^18, 2^20;
//   batch_time  times per device batch: the default and 1, 2, 4, 8;
//   unfused     Z formed inside the product or written to device memory.
// 0 is always a candidate (the library's own choice), so the result is never
// slower than the defaults as timed, and a value replaces the axis's current
// one only when it is more than 0.5 % faster (about the spread of a two-call
// timing), so near-ties keep the defaults.  Each candidate: a context, one call that
// captures and warms the graph, two timed replays (HIP events).  Candidates
// that do not fit in device memory are skipped.  Winners are cached in a JSON
// file, one entry per line, keyed by what decides the product kernel and its
// work: GPU architecture, product path, rows, axes, unique beams, sky flags,
// the source count as a power-of-two bucket, times, channels, precision and
// beam mode, e.g.
//   "gfx950|path3|N700|ax2|nb1|fl4|src2^21|t2|f8|p2|b2": {"ksplit": 0, "batch_time": 0, "src_chunk": 0,
//                                                        "tile": 2, "flags": 0, "ms": 150.1},
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "matvis.h"
#include "internal.h"

namespace {

struct Entry {
    long long ksplit = 0, src_chunk = 0;
    int batch_time = 0, tile = 0, flags = 0;
    double ms = 0;
};

bool field(const std::string &line, const char *name, long long &out) {
    const std::string key = std::string("\"") + name + "\":";
    const size_t p = line.find(key);
    if (p == std::string::npos) return false;
    out = atoll(line.c_str() + p + key.size());
    return true;
}

std::map<std::string, Entry> read_cache(const char *path) {
    std::map<std::string, Entry> out;
    if (!path) return out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        const std::string key = line.substr(q0 + 1, q1 - q0 - 1);
        Entry e;
        long long v = 0;
        bool ok = field(line, "ksplit", e.ksplit) && field(line, "src_chunk", e.src_chunk);
        ok = ok && field(line, "batch_time", v) && (e.batch_time = (int)v, true);
        ok = ok && field(line, "tile", v) && (e.tile = (int)v, true);
        if (field(line, "flags", v)) e.flags = (int)v;
        const size_t pm = line.find("\"ms\":");
        if (pm != std::string::npos) e.ms = atof(line.c_str() + pm + 5);
        if (ok && e.ksplit >= 0 && e.src_chunk >= 0 && e.batch_time >= 0 && e.tile >= 0 && e.ms > 0) out[key] = e;
    }
    return out;
}

bool write_cache(const char *path, const std::map<std::string, Entry> &m) {
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (auto &kv : m) {
            char buf[640];
            snprintf(buf, sizeof buf,
                     "\"%s\": {\"ksplit\": %lld, \"batch_time\": %d, \"src_chunk\": %lld, \"tile\": %d, "
                     "\"flags\": %d, \"ms\": %.4f}%s\n",
                     kv.first.c_str(), kv.second.ksplit, kv.second.batch_time, kv.second.src_chunk, kv.second.tile,
                     kv.second.flags, kv.second.ms, ++i < m.size() ? "," : "");
            f << buf;
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

int prec_of(int32_t p) { return p == MATVIS_FP32 ? mv::P32 : p == MATVIS_BF16X3 ? mv::PB3 : mv::P64; }

// The product path a configuration runs (as matvis_product_path_of reports it),
// from the configuration alone.
int path_of(const matvis_config &c) {
    if (c.precision == MATVIS_FP64 || (c.flags & MATVIS_FLAG_UNFUSED)) return MATVIS_PATH_Z_IN_HBM;
    const int N = c.n_ant * c.n_feed;
    const int Np = (int)((N + 127) / 128 * 128);
    return mv::fused_path(prec_of(c.precision), c.n_feed, c.n_ax, c.n_beam, c.n_ant, Np);
}

}  // namespace

extern "C" matvis_status matvis_autotune(const matvis_config *base, const double *antpos, const int32_t *beam_idx,
                                         const double *freqs, int32_t n_freq, const double *lsts, int32_t n_time,
                                         const double *src_radec, int64_t n_src, const double *src_flux,
                                         const void *beam_grid, void *vis, void *stream, const char *cache_path,
                                         matvis_config *best, double *best_ms, const float *surrogate_params,
                                         double nu_min_hz, double nu_max_hz) {
    if (!base || !best || !best_ms) return MATVIS_EINVAL;
    if (base->beam_mode == MATVIS_BEAM_SURROGATE && !surrogate_params) return MATVIS_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return MATVIS_EHIP;
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    const int path0 = path_of(*base);
    std::ostringstream ks;
    ks << arch << "|path" << path0 << "|N" << base->n_ant * base->n_feed << "|ax" << base->n_ax << "|nb"
       << base->n_beam << "|fl" << (base->flags & MATVIS_FLAG_POLARISED_SKY) << "|src2^"
       << (n_src > 0 ? (int)std::floor(std::log2((double)n_src)) : 0) << "|t" << n_time << "|f" << n_freq << "|p"
       << base->precision << "|b" << base->beam_mode;
    const std::string key = ks.str();
    const int keep = ~(MATVIS_FLAG_UNFUSED | MATVIS_FLAG_NO_GRAPH);
    std::map<std::string, Entry> cache = read_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
        *best = *base;
        best->ksplit = hit->second.ksplit;
        best->batch_time = hit->second.batch_time;
        best->src_chunk = hit->second.src_chunk;
        best->tile = hit->second.tile;
        best->flags = (base->flags & keep) | (hit->second.flags & MATVIS_FLAG_UNFUSED);
        *best_ms = hit->second.ms;
        return MATVIS_OK;
    }

    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MATVIS_EHIP;
    matvis_status last = MATVIS_OK;
    std::map<std::vector<long long>, double> timed;  // candidate -> ms (each timed once)
    auto time_cfg = [&](const matvis_config &c) -> double {
        const std::vector<long long> id = {c.ksplit, c.batch_time, c.src_chunk, c.tile, c.flags};
        auto it = timed.find(id);
        if (it != timed.end()) return it->second;
        double out = 1e300;
        matvis_ctx *ctx = nullptr;
        matvis_status st = matvis_init(&c, &ctx);
        if (st == MATVIS_OK && c.beam_mode == MATVIS_BEAM_SURROGATE)
            st = matvis_set_surrogate(ctx, surrogate_params, nu_min_hz, nu_max_hz);
        if (st == MATVIS_OK)
            st = matvis_simulate(ctx, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux,
                                 beam_grid, vis, stream);
        if (st == MATVIS_OK) st = matvis_finish(ctx);
        float ms = 0.f;
        if (st == MATVIS_OK) {
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 2 && st == MATVIS_OK; r++)
                st = matvis_simulate(ctx, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux,
                                     beam_grid, vis, stream);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = MATVIS_EHIP;
        }
        if (ctx) matvis_destroy(ctx);
        if (st == MATVIS_OK)
            out = ms / 2.0;
        else
            last = st;
        timed[id] = out;
        return out;
    };

    // candidate values per axis (0 = the library's choice)
    const int prec = prec_of(base->precision);
    const bool over_sources = path0 == MATVIS_PATH_SOURCES, three_blocks = path0 == MATVIS_PATH_FUSED_BLOCKS;
    const int64_t kdef = mv::default_ksplit(prec, over_sources, three_blocks);
    std::vector<long long> tiles = {0};  // forming split, bits 0-3
    if (over_sources) tiles.push_back(2);
    if (three_blocks) tiles.insert(tiles.end(), {2, 4});
    std::vector<long long> pair_kernels = {0};  // block-pair kernel, bit 4 (BF16X3, more than one block)
    if (over_sources && prec == mv::PB3 && base->n_ant > 128) pair_kernels.push_back(16);
    std::vector<long long> stages = {0};  // stage depth, bit 6 (BF16X3 three-block path)
    if (three_blocks && prec == mv::PB3) stages.push_back(64);
    std::vector<long long> ksplits = {0};
    for (int64_t d : {kdef * 2, kdef * 4, kdef / 2, kdef / 4})
        if (d >= 64 && d % 64 == 0) ksplits.push_back(d);
    std::vector<long long> chunks = {0};
    for (long long c : {1LL << 18, 1LL << 20})
        if (c < n_src) chunks.push_back(c);
    std::vector<long long> tbs = {0};
    for (int tb : {1, 2, 4, 8})
        if (tb <= base->max_time) tbs.push_back(tb);
    std::vector<long long> fuse = {0};
    if (base->precision != MATVIS_FP64) fuse.push_back(MATVIS_FLAG_UNFUSED);

    matvis_config cur = *base;
    cur.ksplit = 0;
    cur.batch_time = 0;
    cur.src_chunk = 0;
    cur.tile = 0;
    cur.flags = base->flags & keep;
    double cur_ms = time_cfg(cur);
    struct Axis {
        const std::vector<long long> *vals;
        std::function<void(matvis_config &, long long)> set;
    };
    const std::vector<Axis> axes = {
        {&pair_kernels, [](matvis_config &c, long long v) { c.tile = (c.tile & ~16) | (int32_t)v; }},
        {&tiles, [](matvis_config &c, long long v) { c.tile = (c.tile & ~15) | (int32_t)v; }},
        {&stages, [](matvis_config &c, long long v) { c.tile = (c.tile & ~64) | (int32_t)v; }},
        {&ksplits, [](matvis_config &c, long long v) { c.ksplit = v; }},
        {&chunks, [](matvis_config &c, long long v) { c.src_chunk = v; }},
        {&tbs, [](matvis_config &c, long long v) { c.batch_time = (int32_t)v; }},
        {&fuse, [](matvis_config &c, long long v) { c.flags = (c.flags & ~(MATVIS_FLAG_UNFUSED | MATVIS_FLAG_NO_GRAPH)) | (int32_t)v; }},
    };
    // a candidate replaces the current choice only when it is faster by more than
    // the run-to-run spread of a two-call timing (~0.5 %), so ties keep the defaults
    constexpr double kMargin = 0.995;
    for (const Axis &ax : axes)
        for (long long v : *ax.vals) {
            matvis_config c = cur;
            ax.set(c, v);
            const double ms = time_cfg(c);
            if (ms < cur_ms * kMargin) {
                cur_ms = ms;
                cur = c;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cur_ms >= 1e300) return last != MATVIS_OK ? last : MATVIS_ENOMEM;
    *best = cur;
    best->flags = (base->flags & keep) | (cur.flags & MATVIS_FLAG_UNFUSED);
    *best_ms = cur_ms;
    if (cache_path) {
        Entry e;
        e.ksplit = cur.ksplit;
        e.batch_time = cur.batch_time;
        e.src_chunk = cur.src_chunk;
        e.tile = cur.tile;
        e.flags = cur.flags & MATVIS_FLAG_UNFUSED;
        e.ms = cur_ms;
        cache[key] = e;
        write_cache(cache_path, cache);
    }
    return MATVIS_OK;
}
