// Autotuner for the batched product (matvis_autotune in include/matvis.h).
//
// The search space is small and discrete, so it is searched exhaustively on
// the caller's own inputs: for each candidate (k-split, times per batch,
// fused or unfused Z; 0 for the library's own choice) a context is created,
// one call captures and warms the graph, and two replays are timed with HIP
// events.  Candidates that do not
// fit in device memory are skipped.  Winners are cached in a JSON file, one
// entry per line:
//   "gfx950|N256|ax2|src50000|t32|f16|p2|b1": {"ksplit": 4096, "batch_time": 8, "flags": 0, "ms": 23.1},
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "matvis.h"
#include "internal.h"

namespace {

struct Entry {
    long long ksplit = 0;
    int batch_time = 0, flags = 0;
    double ms = 0;
};

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
        const char *p;
        bool has_k = false, has_t = false;  // 0 is a valid value: the library's own choice
        if ((p = strstr(line.c_str(), "\"ksplit\":"))) e.ksplit = atoll(p + 9), has_k = true;
        if ((p = strstr(line.c_str(), "\"batch_time\":"))) e.batch_time = atoi(p + 13), has_t = true;
        if ((p = strstr(line.c_str(), "\"flags\":"))) e.flags = atoi(p + 8);
        if ((p = strstr(line.c_str(), "\"ms\":"))) e.ms = atof(p + 5);
        if (has_k && has_t && e.ksplit >= 0 && e.batch_time >= 0 && e.ms > 0) out[key] = e;
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
            char buf[512];
            snprintf(buf, sizeof buf, "\"%s\": {\"ksplit\": %lld, \"batch_time\": %d, \"flags\": %d, \"ms\": %.4f}%s\n",
                     kv.first.c_str(), kv.second.ksplit, kv.second.batch_time, kv.second.flags, kv.second.ms,
                     ++i < m.size() ? "," : "");
            f << buf;
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" matvis_status matvis_autotune(const matvis_config *base, const double *antpos, const int32_t *beam_idx,
                                         const double *freqs, int32_t n_freq, const double *lsts, int32_t n_time,
                                         const double *src_radec, int64_t n_src, const double *src_flux,
                                         const void *beam_grid, void *vis, void *stream, const char *cache_path,
                                         matvis_config *best, double *best_ms) {
    if (!base || !best || !best_ms) return MATVIS_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return MATVIS_EHIP;
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::ostringstream ks;
    ks << arch << "|N" << base->n_ant * base->n_feed << "|ax" << base->n_ax << "|src" << n_src << "|t" << n_time
       << "|f" << n_freq << "|p" << base->precision << "|b" << base->beam_mode;
    const std::string key = ks.str();
    std::map<std::string, Entry> cache = read_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
        *best = *base;
        best->ksplit = hit->second.ksplit;
        best->batch_time = hit->second.batch_time;
        best->flags = (base->flags & ~MATVIS_FLAG_UNFUSED) | (hit->second.flags & MATVIS_FLAG_UNFUSED);
        *best_ms = hit->second.ms;
        return MATVIS_OK;
    }

    // 0 is the library's own choice (per precision and product path), so the
    // winner is never slower than the defaults; the other k-splits are at most
    // the defaults of the fused paths, so never less accurate than them
    std::vector<long long> ksplits;
    if (base->precision == MATVIS_FP64)
        ksplits = {0, 4096, 16384};
    else if (base->precision == MATVIS_FP32)
        ksplits = {0, 1024, 2048};
    else
        ksplits = {0, 2048, 4096, 8192};
    std::vector<int> tbs = {0};
    for (int tb : {2, 4, 8})
        if (tb <= base->max_time) tbs.push_back(tb);
    std::vector<int> fuse = {0};
    if (base->precision != MATVIS_FP64) fuse.push_back(MATVIS_FLAG_UNFUSED);

    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MATVIS_EHIP;
    double bms = 1e300;
    matvis_config bcfg = *base;
    matvis_status last = MATVIS_OK;
    for (long long ksp : ksplits)
        for (int tb : tbs)
            for (int fl : fuse) {
                matvis_config c = *base;
                c.ksplit = ksp;
                c.batch_time = tb;
                c.flags = (base->flags & ~(MATVIS_FLAG_UNFUSED | MATVIS_FLAG_NO_GRAPH)) | fl;
                matvis_ctx *ctx = nullptr;
                matvis_status st = matvis_init(&c, &ctx);
                if (st != MATVIS_OK) {
                    last = st;
                    continue;
                }
                st = matvis_simulate(ctx, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src, src_flux,
                                     beam_grid, vis, stream);
                if (st == MATVIS_OK) st = matvis_finish(ctx);
                float ms = 0.f;
                if (st == MATVIS_OK) {
                    (void)hipEventRecord(e0, s);
                    for (int r = 0; r < 2 && st == MATVIS_OK; r++)
                        st = matvis_simulate(ctx, antpos, beam_idx, freqs, n_freq, lsts, n_time, src_radec, n_src,
                                             src_flux, beam_grid, vis, stream);
                    (void)hipEventRecord(e1, s);
                    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                        st = MATVIS_EHIP;
                }
                matvis_destroy(ctx);
                if (st != MATVIS_OK) {
                    last = st;
                    continue;
                }
                if (ms / 2.0 < bms) {
                    bms = ms / 2.0;
                    bcfg = c;
                    bcfg.flags = (base->flags & ~MATVIS_FLAG_UNFUSED) | fl;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (bms >= 1e300) return last != MATVIS_OK ? last : MATVIS_ENOMEM;
    *best = bcfg;
    *best_ms = bms;
    if (cache_path) {
        Entry e;
        e.ksplit = bcfg.ksplit;
        e.batch_time = bcfg.batch_time;
        e.flags = bcfg.flags & MATVIS_FLAG_UNFUSED;
        e.ms = bms;
        cache[key] = e;
        write_cache(cache_path, cache);
    }
    return MATVIS_OK;
}
