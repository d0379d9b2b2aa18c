// sw_autotune.hip -- tile-shape and persistent-grid autotuner.
//
// Results never depend on the tile shape or the grid (every union hooks to
// the smaller root), so the tuner is free to pick whatever runs fastest.  For
// each (dim, size class = floor(log2 L)) present in a handle it times every
// compiled tile shape on a scratch lattice with the same parameters, and for
// the persistent engine the workgroups per CU; choices are cached as JSON.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sw_runtime.hpp"

namespace sw {

struct TuneKey {
    int dim, lclass;
    bool operator<(const TuneKey& o) const { return dim != o.dim ? dim < o.dim : lclass < o.lclass; }
};

static int size_class(int L)
{
    int c = 0;
    while ((2 << c) <= L) ++c;
    return c;
}

static std::string key_string(const TuneKey& k)
{
    char buf[64];
    snprintf(buf, sizeof(buf), "gfx950:d%d:l%d", k.dim, k.lclass);
    return buf;
}

// minimal reader for the cache this file writes: {"key": {"shape": s, "ms": t}, ...}
static std::map<std::string, int> read_cache(const char* path)
{
    std::map<std::string, int> out;
    if (!path) return out;
    FILE* f = fopen(path, "rb");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
    fclose(f);
    size_t pos = 0;
    while ((pos = txt.find("\"gfx950:", pos)) != std::string::npos) {
        const size_t end = txt.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = txt.substr(pos + 1, end - pos - 1);
        const size_t sp = txt.find("\"shape\":", end);
        if (sp == std::string::npos) break;
        out[key] = atoi(txt.c_str() + sp + 8);
        pos = end + 1;
    }
    return out;
}

static void write_cache(const char* path, const std::map<std::string, std::pair<int, double>>& entries)
{
    if (!path) return;
    FILE* f = fopen(path, "wb");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : entries) {
        fprintf(f, "  \"%s\": {\"shape\": %d, \"ms_per_sweep\": %.6f}%s\n", kv.first.c_str(), kv.second.first,
                kv.second.second, (++i < entries.size()) ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
}

// milliseconds per sweep of a scratch single-replica lattice with this shape
static int time_shape(const sw_params& prm, int shape, int sweeps, hipStream_t stream, double* ms_out)
{
    sw_params p = prm;
    p.flags &= ~(uint32_t)SW_RECORD_SERIES;
    sw_lattice* h = nullptr;
    int rc = sw_init(&p, 1, -1, stream, &h);
    if (rc) return rc;
    rc = sw_set_tile_shape(h, 0, shape);
    if (!rc) rc = sw_sweep(h, 1);                      // warm-up
    if (!rc) rc = handle_sync(h);
    hipEvent_t a = nullptr, b = nullptr;
    if (!rc && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) rc = fail(SW_EHIP, "event");
    if (!rc) {
        hipEventRecord(a, h->stream);
        rc = sw_sweep(h, sweeps);
        hipEventRecord(b, h->stream);
    }
    if (!rc) rc = handle_sync(h);
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = fail(SW_EHIP, "event timing");
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    sw_free(h);
    if (!rc) *ms_out = ms / sweeps;
    return rc;
}

}  // namespace sw

using namespace sw;

extern "C" int sw_autotune(sw_lattice* h, int32_t sweeps, const char* cache_path)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (sweeps < 1) return fail(SW_EINVAL, "need at least one timed sweep");
    int rc = sync_mirror(h);
    if (rc) return rc;
    std::map<TuneKey, int> rep_of;                       // representative replica per class
    for (size_t r = 0; r < h->reps.size(); ++r) {
        const TuneKey k{h->reps[r].h.dim, size_class(h->reps[r].h.L)};
        if (!rep_of.count(k) || h->reps[r].h.L > h->reps[rep_of[k]].h.L) rep_of[k] = (int)r;
    }
    auto cached = read_cache(cache_path);
    std::map<std::string, std::pair<int, double>> out;
    std::map<TuneKey, int> choice;
    for (auto& kv : rep_of) {
        const std::string ks = key_string(kv.first);
        if (cached.count(ks) && cached[ks] >= 0 && cached[ks] < shape_count(kv.first.dim)) {
            choice[kv.first] = cached[ks];
            out[ks] = {cached[ks], -1.0};
            continue;
        }
        const sw_params& prm = h->reps[kv.second].prm;
        int best = default_shape(prm.dim);
        double best_ms = 1e30;
        for (int s = 0; s < shape_count(prm.dim); ++s) {
            double ms = 0;
            rc = time_shape(prm, s, sweeps, h->stream, &ms);
            if (rc) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = s;
            }
        }
        choice[kv.first] = best;
        out[ks] = {best, best_ms};
    }
    for (size_t r = 0; r < h->reps.size(); ++r) {
        const TuneKey k{h->reps[r].h.dim, size_class(h->reps[r].h.L)};
        rc = sw_set_tile_shape(h, (int32_t)r, choice[k]);
        if (rc) return rc;
    }
    // persistent engine: workgroups per CU, timed on a scratch copy of all replicas
    if (h->reps.size() > 1) {
        const int limit = engine_grid_limit();
        if (limit > 0) {
            const int cus = device_cu_count();
            std::vector<sw_params> ps;
            for (auto& r : h->reps) {
                sw_params p = r.prm;
                p.flags &= ~(uint32_t)SW_RECORD_SERIES;
                ps.push_back(p);
            }
            sw_lattice* s = nullptr;
            rc = sw_init(ps.data(), (int32_t)ps.size(), -1, h->stream, &s);
            if (rc) return rc;
            for (size_t r = 0; r < ps.size() && !rc; ++r) rc = sw_set_tile_shape(s, (int32_t)r, h->reps[r].h.shape);
            s->mode = SW_MODE_BATCHED;
            double best_ms = 1e30;
            int best_cap = 0;
            for (int cap : {limit, std::max(cus, limit / 2), std::max(cus, limit / 4)}) {
                if (rc) break;
                s->engine_grid_cap = cap;
                rc = sw_sweep(s, 1);                      // capture + warm-up
                if (!rc) rc = handle_sync(s);
                if (rc) break;
                hipEvent_t a = nullptr, b = nullptr;
                hipEventCreate(&a);
                hipEventCreate(&b);
                hipEventRecord(a, s->stream);
                rc = sw_sweep(s, 1);
                hipEventRecord(b, s->stream);
                if (!rc) rc = handle_sync(s);
                float ms = 0.f;
                if (!rc) hipEventElapsedTime(&ms, a, b);
                hipEventDestroy(a);
                hipEventDestroy(b);
                if (!rc && ms < best_ms) {
                    best_ms = ms;
                    best_cap = cap;
                }
            }
            sw_free(s);
            if (rc) return rc;
            h->engine_grid_cap = best_cap;
        }
    }
    write_cache(cache_path, out);
    return SW_OK;
}
