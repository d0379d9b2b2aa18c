// sw_autotune.hip -- tile-shape, merge-schedule and batched-grid autotuner.
//
// Results never depend on the tile shape, the border-merge width or the grid
// (every union hooks to the smaller root), so the tuner is free to pick
// whatever runs fastest.
//   one replica:   every compiled tile shape, each with both border-merge
//                  widths (64 and 256 threads per tile), is timed with plain
//                  launches on a scratch lattice with the same parameters
//                  and state;
//   many replicas: every batched variant (a 2D and a 3D shape), both merge
//                  widths and four grid sizes of the phase-kernel graph, and
//                  the persistent engine, are timed on a scratch copy of all
//                  replicas (parameters and state) in batched mode.
// Choices are cached as JSON keyed by (arch, dim, size class = floor(log2 L))
// for single lattices and by (arch, "batch", replica count, total sites) for
// batches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sw_runtime.hpp"

namespace sw {

static int size_class(int L)
{
    int c = 0;
    while ((2 << c) <= L) ++c;
    return c;
}

struct Choice {
    int shape, grid, merge, engine;
    double ms;
};

// minimal reader for the cache this file writes:
// {"key": {"shape": s, "grid": g, "merge": m, "engine": e, ...}, ...}; an
// entry without "merge" or "engine" takes the default (0)
static std::map<std::string, Choice> read_cache(const char* path)
{
    std::map<std::string, Choice> out;
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
        const size_t close = txt.find('}', end);
        const size_t sp = txt.find("\"shape\":", end);
        const size_t gp = txt.find("\"grid\":", end);
        if (sp == std::string::npos || gp == std::string::npos || close == std::string::npos) break;
        const size_t mp = txt.find("\"merge\":", end);
        const int merge = (mp != std::string::npos && mp < close) ? atoi(txt.c_str() + mp + 8) : 0;
        const size_t ep = txt.find("\"engine\":", end);
        const int engine = (ep != std::string::npos && ep < close) ? atoi(txt.c_str() + ep + 9) : 0;
        out[key] = Choice{atoi(txt.c_str() + sp + 8), atoi(txt.c_str() + gp + 7), merge, engine, -1.0};
        pos = end + 1;
    }
    return out;
}

static void write_cache(const char* path, const std::map<std::string, Choice>& entries)
{
    if (!path) return;
    std::map<std::string, Choice> all = read_cache(path);
    for (auto& kv : entries) all[kv.first] = kv.second;
    FILE* f = fopen(path, "wb");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : all) {
        fprintf(f, "  \"%s\": {\"shape\": %d, \"grid\": %d, \"merge\": %d, \"engine\": %d, \"ms_per_sweep\": %.6f}%s\n",
                kv.first.c_str(), kv.second.shape, kv.second.grid, kv.second.merge, kv.second.engine, kv.second.ms,
                (++i < all.size()) ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
}

// scratch replica r of s starts from the current spins and sweep counter of
// replica src of h (cluster sizes, and so the cost of a sweep, depend on the
// state: a random start is not representative)
static int copy_state(sw_lattice* s, int r, const sw_lattice* h, int src)
{
    const SwRep& from = h->reps[src].h;
    SwRep& to = s->reps[r].h;
    hipError_t e = hipMemcpyAsync(to.spins, from.spins, spin_bytes(from), hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "copying spins to the tuning lattice");
    to.sweep = from.sweep;
    to.thr = from.thr;
    to.p = from.p;
    return push_desc(s, r);
}

// milliseconds per sweep of `sweeps` sweeps on handle s, after an untimed call
// of the same size (which, in batched mode, builds the graph the timed call
// replays, so that graph capture stays outside the timed region)
static int time_sweeps(sw_lattice* s, int sweeps, double* ms_out)
{
    int rc = sw_sweep(s, sweeps);
    if (!rc) rc = handle_sync(s);
    if (rc) return rc;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) hipEventDestroy(a);
        return fail(SW_EHIP, "event creation failed");
    }
    hipEventRecord(a, s->stream);
    rc = sw_sweep(s, sweeps);
    hipEventRecord(b, s->stream);
    if (!rc) rc = handle_sync(s);
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = fail(SW_EHIP, "event timing failed");
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (!rc) *ms_out = ms / sweeps;
    return rc;
}

static int tune_single(sw_lattice* h, int32_t sweeps, const char* cache_path)
{
    ReplicaH& rep = h->reps[0];
    char key[64];
    snprintf(key, sizeof(key), "gfx950:d%d:l%d", rep.h.dim, size_class(rep.h.L));
    auto cached = read_cache(cache_path);
    auto it = cached.find(key);
    if (it != cached.end() && it->second.shape >= 0 && it->second.shape < shape_count(rep.h.dim)) {
        int rc = sw_set_tile_shape(h, 0, it->second.shape);
        return rc ? rc : sw_set_merge_width(h, it->second.merge);
    }
    sw_params p = rep.prm;
    p.flags &= ~(uint32_t)SW_RECORD_SERIES;
    int best = default_shape(p.dim), best_merge = 0;
    double best_ms = 1e30;
    for (int shape = 0; shape < shape_count(p.dim); ++shape) {
        sw_lattice* s = nullptr;
        int rc = sw_init(&p, 1, -1, h->stream, &s);
        if (!rc) rc = sw_set_tile_shape(s, 0, shape);
        for (int merge : {64, 256}) {
            if (rc) break;
            rc = copy_state(s, 0, h, 0);
            if (!rc) rc = sw_set_merge_width(s, merge);
            double ms = 0;
            if (!rc) rc = time_sweeps(s, sweeps, &ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best = shape;
                best_merge = merge;
            }
        }
        if (s) sw_free(s);
        if (rc) return rc;
    }
    std::map<std::string, Choice> out;
    out[key] = Choice{best, 0, best_merge, 0, best_ms};
    write_cache(cache_path, out);
    int rc = sw_set_tile_shape(h, 0, best);
    return rc ? rc : sw_set_merge_width(h, best_merge);
}

static int tune_batch(sw_lattice* h, int32_t sweeps, const char* cache_path)
{
    uint64_t total = 0;
    for (auto& r : h->reps) total += r.h.N;
    char key[96];
    snprintf(key, sizeof(key), "gfx950:batch:r%zu:n%llu", h->reps.size(), (unsigned long long)total);
    int best_v = 0, best_grid = 0, best_merge = 0, best_engine = SW_ENGINE_GRAPH;
    double best_ms = 1e30;
    auto cached = read_cache(cache_path);
    auto it = cached.find(key);
    if (it != cached.end() && it->second.shape >= 0 && it->second.shape < shape_count(2)) {
        best_v = it->second.shape;
        best_grid = it->second.grid;
        best_merge = it->second.merge;
        best_engine = it->second.engine == SW_ENGINE_PERSISTENT ? SW_ENGINE_PERSISTENT : SW_ENGINE_GRAPH;
    } else {
        std::vector<sw_params> ps;
        for (auto& r : h->reps) {
            sw_params p = r.prm;
            p.flags &= ~(uint32_t)SW_RECORD_SERIES;
            ps.push_back(p);
        }
        for (int v = 0; v < shape_count(2); ++v) {
            sw_lattice* s = nullptr;
            int rc = sw_init(ps.data(), (int32_t)ps.size(), -1, h->stream, &s);
            for (size_t r = 0; r < ps.size() && !rc; ++r) rc = sw_set_tile_shape(s, (int32_t)r, v);
            if (!rc) s->mode = SW_MODE_BATCHED;
            // every candidate starts from the batch's own state: the cost of a
            // sweep changes as the replicas equilibrate, so candidates timed one
            // after the other on a running copy would favour the later ones
            auto restart = [&]() {
                int e = 0;
                for (size_t r = 0; r < ps.size() && !e; ++r) e = copy_state(s, (int)r, h, (int)r);
                return e;
            };
            for (int merge : {64, 256}) {
                for (int per_cu : {0, 4, 8, 16}) {
                    if (!rc) rc = restart();
                    if (rc) break;
                    s->batch_per_cu = per_cu;
                    s->merge_width = merge;
                    double ms = 0;
                    rc = time_sweeps(s, sweeps, &ms);
                    if (!rc && ms < best_ms) {
                        best_ms = ms;
                        best_v = v;
                        best_grid = per_cu;
                        best_merge = merge;
                        best_engine = SW_ENGINE_GRAPH;
                    }
                }
            }
            if (!rc) rc = restart();
            if (!rc) {
                // the persistent engine, with as many workgroups as fit
                s->batch_engine = SW_ENGINE_PERSISTENT;
                s->batch_per_cu = 0;
                s->merge_width = 0;
                double ms = 0;
                rc = time_sweeps(s, sweeps, &ms);
                if (!rc && ms < best_ms) {
                    best_ms = ms;
                    best_v = v;
                    best_grid = 0;
                    best_merge = 0;
                    best_engine = SW_ENGINE_PERSISTENT;
                }
            }
            if (s) sw_free(s);
            if (rc) return rc;
        }
        std::map<std::string, Choice> out;
        out[key] = Choice{best_v, best_grid, best_merge, best_engine, best_ms};
        write_cache(cache_path, out);
    }
    for (size_t r = 0; r < h->reps.size(); ++r) {
        int rc = sw_set_tile_shape(h, (int32_t)r, best_v);
        if (rc) return rc;
    }
    if (best_grid >= 0) h->batch_per_cu = best_grid;
    h->batch_engine = best_engine;
    return sw_set_merge_width(h, best_merge);
}

}  // namespace sw

using namespace sw;

extern "C" int sw_autotune(sw_lattice* h, int32_t sweeps, const char* cache_path)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (sweeps < 1) return fail(SW_EINVAL, "need at least one timed sweep");
    if (hipSetDevice(h->device) != hipSuccess) return fail(SW_EHIP, "hipSetDevice failed");
    int rc = sync_mirror(h);
    if (rc) return rc;
    return h->reps.size() == 1 ? tune_single(h, sweeps, cache_path) : tune_batch(h, sweeps, cache_path);
}
