// sw_runtime.hip -- host runtime and C ABI of libswgpu.so (lattice handles).
//
// A handle owns R replicas.  For each it keeps a host mirror of the device
// descriptor (SwRep), the device buffers, and the bookkeeping of the sweep
// counter and the (E_int, M) series.  Plain mode enqueues the phase kernels
// replica by replica; batched mode replays a hipGraph whose phase kernels
// each run over the work list of every replica's tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sw_api.h"
#include "sw_device.hpp"
#include "sw_internal.hpp"
#include "sw_runtime.hpp"

namespace sw {

static thread_local std::string g_error = "no error";

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(SW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_error.c_str(); }

static int g_cu_count[64];
static uint64_t g_wall_hz[64];

int device_cu_count()
{
    int dev = 0;
    hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (!g_cu_count[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

uint64_t device_wallclock_hz()
{
    int dev = 0;
    hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (!g_wall_hz[dev]) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        g_wall_hz[dev] = (uint64_t)khz * 1000ull;
    }
    return g_wall_hz[dev];
}

uint64_t threshold_from_p(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)std::floor(std::ldexp(p, 32));
}

int validate_params(const sw_params* p)
{
    if (!p) return fail(SW_EINVAL, "null parameters");
    if (p->dim != 2 && p->dim != 3) return fail(SW_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->L < 3) return fail(SW_EINVAL, "L must be >= 3 (got %d)", p->L);
    uint64_t n = 1;
    for (int d = 0; d < p->dim; ++d) n *= (uint64_t)p->L;
    if (n >= (1ull << 31)) return fail(SW_EINVAL, "L^dim must be < 2^31 (int32 labels)");
    if ((uint64_t)p->dim * n >= (1ull << 32)) return fail(SW_EINVAL, "dim*L^dim must be < 2^32 (32-bit link index)");
    if (!(p->J > 0.0) || !std::isfinite(p->J)) return fail(SW_EINVAL, "J must be finite and > 0 (ferromagnet)");
    if (p->p_bond < 0.0) {
        if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(SW_EINVAL, "T must be finite and > 0");
    } else if (!(p->p_bond <= 1.0)) {
        return fail(SW_EINVAL, "p_bond must be in [0,1] or negative");
    }
    if (p->flags & ~(uint32_t)(SW_RECORD_SERIES | SW_KEEP_LABELS | SW_PCC | SW_BITPACK | SW_OPEN | SW_PCC_WIND))
        return fail(SW_EINVAL, "unknown flags");
    if ((p->flags & SW_PCC_WIND) && (!(p->flags & SW_PCC) || (p->flags & SW_OPEN)))
        return fail(SW_EINVAL, "the topological rule needs SW_PCC on a periodic box");
    if (p->flags & SW_PCC) {
        if (!(p->pcc_dp0 > 0.0) || !std::isfinite(p->pcc_dp0)) return fail(SW_EINVAL, "pcc_dp0 must be > 0");
        if (p->pcc_halve_every == 0) return fail(SW_EINVAL, "pcc_halve_every must be > 0");
    }
    return SW_OK;
}

uint64_t nsites_of(const sw_params* p)
{
    uint64_t n = 1;
    for (int d = 0; d < p->dim; ++d) n *= (uint64_t)p->L;
    return n;
}

// default tile shape per dimension (the autotuner may replace it)
int default_shape(int dim) { return dim == 2 ? 0 : 0; }

void fill_geometry(SwRep& h, int shape)
{
    int tx = 0, ty = 0, tz = 0;
    shape_extents(h.dim, shape, &tx, &ty, &tz);
    h.shape = shape;
    h.tx = tx;
    h.ty = ty;
    h.tz = tz;
    h.ntx = (h.L + tx - 1) / tx;
    h.nty = (h.L + ty - 1) / ty;
    h.ntz = (h.dim == 3) ? (h.L + tz - 1) / tz : 1;
    h.ntiles = h.ntx * h.nty * h.ntz;
    h.xwords = shape_xwords(h.dim, shape);
    h.fbw = shape_fbw(h.dim, shape);
    h.ft = shape_ft(h.dim, shape);
}

// per-tile buffers: crossing bits, border-root bitmaps and their flip bits,
// face ranks, the border merge's slots (not with the topological rule), and
// for PCC the coverage entries of the border roots (and, for the extension
// rule or the open box, the ranks of the bitmap words)
static uint64_t tile_bytes(const SwRep& h, uint32_t flags)
{
    const uint64_t nt = (uint64_t)h.ntiles;
    const bool pcc = (flags & FLAG_PCC) != 0, wind = (flags & FLAG_WIND) != 0;
    uint64_t b = nt * (uint64_t)h.xwords * 4 + 2 * nt * (uint64_t)h.fbw * 4 + nt * 2 * (uint64_t)h.ft * 2;
    if (!wind) b += nt * 2 * (uint64_t)h.ft * 8;
    if (pcc) b += nt * 2 * (uint64_t)h.ft * 16;
    if (pcc && !wind) b += nt * (uint64_t)h.fbw * 2;
    return b;
}

// bytes of a replica's spin array: N int8, or ceil(N/32) words bit-packed
size_t spin_bytes(const SwRep& h)
{
    return (h.flags & FLAG_BITPACK) ? ((size_t)h.N + 31) / 32 * 4 : (size_t)h.N;
}

uint64_t footprint_bytes(const sw_params* p, int shape)
{
    const uint64_t n = nsites_of(p);
    SwRep h{};
    h.dim = p->dim;
    h.L = p->L;
    fill_geometry(h, shape);
    uint64_t b = 2 * ((n + 3) & ~(uint64_t)3);              // lab16 (whole groups of 4 sites)
    b += (p->flags & SW_BITPACK) ? (n + 31) / 32 * 4 : n;    // spins
    if (p->flags & SW_KEEP_LABELS) b += 8 * n;               // lab32, the border roots' cluster roots
    if (p->flags & SW_PCC_WIND) b += 8 * n;                  // parents with sheet offsets
    uint32_t fl = 0;
    if (p->flags & SW_PCC) fl |= FLAG_PCC;
    if (p->flags & SW_PCC_WIND) fl |= FLAG_WIND;
    b += tile_bytes(h, fl);                                  // crossing bits, bitmaps, face ranks, slots, coverage
    b += 64;                                                 // accumulators
    if (p->flags & SW_PCC) {
        const uint64_t L = (uint64_t)p->L;
        const uint64_t ns = (p->dim == 3) ? L * L : L;
        b += (uint64_t)p->dim * n * 8;                       // candidate marks
        b += (uint64_t)p->dim * ns * ((L + 31) / 32) * 4;    // coverage bitmaps
    }
    return b;
}

}  // namespace sw

namespace sw {

// ---------------------------------------------------------------------------
// Handle internals.
// ---------------------------------------------------------------------------
static int dmalloc(void** p, size_t bytes, const char* what)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SW_ENOMEM, "hipMalloc(%zu) for %s failed: %s", bytes, what, hipGetErrorString(e));
    }
    return SW_OK;
}

static void dfree(void* p)
{
    if (p) (void)hipFree(p);
}

static void free_tile_buffers(SwRep& h)
{
    dfree(h.xbits);
    dfree(h.fbits);
    dfree(h.bflip);
    dfree(h.face);
    dfree(h.dpar);
    dfree(h.cov);
    dfree(h.fpre);
    h.xbits = h.fbits = h.bflip = nullptr;
    h.face = h.fpre = nullptr;
    h.cov = h.dpar = nullptr;
}

// the per-tile buffers of a descriptor whose geometry and flags are filled in
static int alloc_tile_buffers(SwRep& h)
{
    const size_t nt = (size_t)h.ntiles;
    const bool wind = (h.flags & FLAG_WIND) != 0;
    h.xbits = h.fbits = h.bflip = nullptr;
    h.face = h.fpre = nullptr;
    h.cov = h.dpar = nullptr;
    h.nslots = (uint32_t)(nt * 2 * (size_t)h.ft);
    int rc = dmalloc((void**)&h.xbits, nt * h.xwords * 4, "crossing bits");
    if (!rc) rc = dmalloc((void**)&h.fbits, nt * h.fbw * 4, "border bitmaps");
    if (!rc) rc = dmalloc((void**)&h.bflip, nt * h.fbw * 4, "border flip bits");
    if (!rc) rc = dmalloc((void**)&h.face, nt * 2 * h.ft * 2, "face ranks");
    if (!rc && !wind) rc = dmalloc((void**)&h.dpar, (size_t)h.nslots * 8, "border-merge slots");
    if (!rc && (h.flags & FLAG_PCC)) rc = dmalloc((void**)&h.cov, nt * 2 * h.ft * 16, "coverage entries");
    if (!rc && (h.flags & FLAG_PCC) && !wind) rc = dmalloc((void**)&h.fpre, nt * h.fbw * 2, "border-root ranks");
    if (rc) free_tile_buffers(h);
    return rc;
}

void replica_free(ReplicaH& r)
{
    if (r.own_spins) dfree(r.h.spins);
    dfree(r.h.lab16);
    dfree(r.h.par);
    dfree(r.h.par64);
    dfree(r.h.lab32);
    free_tile_buffers(r.h);
    dfree(r.h.series);
    dfree(r.h.acc);
    dfree(r.h.cand);
    dfree(r.h.bmp);
    dfree(r.h.pflag);
    dfree(r.h.perc_trace);
    dfree(r.h.p_trace);
    r.h.spins = nullptr;
    r.h.lab16 = nullptr;
    r.h.par = r.h.lab32 = r.h.pflag = r.h.perc_trace = nullptr;
    r.h.par64 = nullptr;
    r.h.bmp = nullptr;
    r.h.series = r.h.acc = nullptr;
    r.h.cand = nullptr;
    r.h.p_trace = nullptr;
}

int replica_alloc(ReplicaH& r, const sw_params* p, int shape, hipStream_t stream)
{
    r.prm = *p;
    SwRep& h = r.h;
    memset(&h, 0, sizeof(h));
    h.dim = p->dim;
    h.L = p->L;
    h.N = (uint32_t)nsites_of(p);
    fill_geometry(h, shape);
    h.flags = 0;
    if (p->flags & SW_RECORD_SERIES) h.flags |= FLAG_SERIES;
    if (p->flags & SW_KEEP_LABELS) h.flags |= FLAG_KEEP;
    if (p->flags & SW_PCC) h.flags |= FLAG_PCC;
    if (p->flags & SW_BITPACK) h.flags |= FLAG_BITPACK;
    if (p->flags & SW_OPEN) h.flags |= FLAG_OPEN;
    if (p->flags & SW_PCC_WIND) h.flags |= FLAG_WIND;
    h.seed = p->seed;
    h.p = (p->p_bond < 0.0) ? -std::expm1(-2.0 * p->J / p->T) : p->p_bond;
    h.thr = threshold_from_p(h.p);
    h.dp0 = p->pcc_dp0;
    h.halve_every = p->pcc_halve_every ? p->pcc_halve_every : 1;
    h.sweep = 0;
    h.limit = 0xFFFFFFFFu;
    h.measured = 0;
    h.active = 1;
    const size_t n = h.N;
    int rc;
    r.own_spins = true;
    if ((rc = dmalloc((void**)&h.spins, spin_bytes(h), "spins"))) goto bad;
    // (rounded up to whole groups of 4 sites: the flip kernel loads 4 labels
    // from any 4-site-aligned position below N)
    if ((rc = dmalloc((void**)&h.lab16, 2 * ((n + 3) & ~(size_t)3), "tile labels"))) goto bad;
    if (h.flags & FLAG_WIND)
        if ((rc = dmalloc((void**)&h.par64, 8 * n, "union-find parents with sheet offsets"))) goto bad;
    if (h.flags & FLAG_KEEP) {
        if ((rc = dmalloc((void**)&h.par, 4 * n, "cluster roots of the border roots"))) goto bad;
        if ((rc = dmalloc((void**)&h.lab32, 4 * n, "labels"))) goto bad;
    }
    if ((rc = alloc_tile_buffers(h))) goto bad;
    if ((rc = dmalloc((void**)&h.acc, 64, "accumulators"))) goto bad;
    if (h.flags & FLAG_SERIES) {
        h.series_cap = p->series_cap ? p->series_cap : 1024;
        if ((rc = dmalloc((void**)&h.series, (size_t)h.series_cap * 16, "series"))) goto bad;
        if (hipMemsetAsync(h.series, 0, (size_t)h.series_cap * 16, stream) != hipSuccess) {
            rc = fail(SW_EHIP, "clearing the series failed");
            goto bad;
        }
    }
    if (h.flags & FLAG_PCC) {
        const size_t L = (size_t)h.L;
        const size_t ns = (h.dim == 3) ? L * L : L;
        const size_t bmp_bytes = (size_t)h.dim * ns * ((L + 31) / 32) * 4;
        if ((rc = dmalloc((void**)&h.cand, (size_t)h.dim * n * 8, "percolation candidates"))) goto bad;
        if ((rc = dmalloc((void**)&h.bmp, bmp_bytes, "coverage bitmaps"))) goto bad;
        if ((rc = dmalloc((void**)&h.pflag, 16, "percolation flag"))) goto bad;
        h.trace_cap = p->series_cap ? p->series_cap : 1024;
        if ((rc = dmalloc((void**)&h.perc_trace, (size_t)h.trace_cap * 4, "percolation trace"))) goto bad;
        if ((rc = dmalloc((void**)&h.p_trace, (size_t)h.trace_cap * 8, "p trace"))) goto bad;
        if (hipMemsetAsync(h.cand, 0, (size_t)h.dim * n * 8, stream) != hipSuccess ||
            hipMemsetAsync(h.bmp, 0, bmp_bytes, stream) != hipSuccess ||
            hipMemsetAsync(h.pflag, 0, 16, stream) != hipSuccess) {
            rc = fail(SW_EHIP, "clearing the percolation buffers failed");
            goto bad;
        }
    }
    return SW_OK;
bad:
    replica_free(r);
    return rc;
}

// the N spins of a replica as int8 +1/-1 in host memory (a bit-packed array
// is unpacked here; the device holds only the packed words)
int read_spins(const SwRep& m, int8_t* host_buf)
{
    if (!(m.flags & FLAG_BITPACK)) {
        hipError_t e = hipMemcpy(host_buf, m.spins, m.N, hipMemcpyDeviceToHost);
        return e == hipSuccess ? SW_OK : hip_fail(e, "reading spins");
    }
    std::vector<uint32_t> w(((size_t)m.N + 31) / 32);
    hipError_t e = hipMemcpy(w.data(), m.spins, w.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading spins");
    for (size_t i = 0; i < m.N; ++i) host_buf[i] = ((w[i >> 5] >> (i & 31)) & 1u) ? 1 : -1;
    return SW_OK;
}

static int write_spins(const SwRep& m, const int8_t* host_buf)
{
    if (!(m.flags & FLAG_BITPACK)) {
        hipError_t e = hipMemcpy(m.spins, host_buf, m.N, hipMemcpyHostToDevice);
        return e == hipSuccess ? SW_OK : hip_fail(e, "writing spins");
    }
    std::vector<uint32_t> w(((size_t)m.N + 31) / 32, 0u);
    for (size_t i = 0; i < m.N; ++i)
        if (host_buf[i] > 0) w[i >> 5] |= 1u << (i & 31);
    hipError_t e = hipMemcpy(m.spins, w.data(), w.size() * 4, hipMemcpyHostToDevice);
    return e == hipSuccess ? SW_OK : hip_fail(e, "writing spins");
}

static int check_rep(sw_lattice* h, int32_t r)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (r < 0 || r >= (int32_t)h->reps.size()) return fail(SW_EINVAL, "replica %d out of range", r);
    return SW_OK;
}

static int set_device(sw_lattice* h)
{
    hipError_t e = hipSetDevice(h->device);
    return e == hipSuccess ? SW_OK : hip_fail(e, "hipSetDevice");
}

int handle_sync(sw_lattice* h)
{
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (h->err) {
        int32_t bits = 0;
        e = hipMemcpy(&bits, h->err, sizeof(bits), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the consistency-check word");
        if (bits) {
            const int32_t zero = 0;
            (void)hipMemcpy(h->err, &zero, sizeof(zero), hipMemcpyHostToDevice);
            return fail(SW_EHIP, "device consistency check failed (bits 0x%x): results of the last sweeps are invalid",
                        (unsigned)bits);
        }
    }
    return SW_OK;
}

// bring the host mirrors up to date after device-side updates (batched
// sweeps, PCC feedback); waits for the stream and checks the error word
int sync_mirror(sw_lattice* h)
{
    int rc = handle_sync(h);
    if (rc) return rc;
    if (!h->mirror_stale) return SW_OK;
    std::vector<SwRep> tmp(h->reps.size());
    hipError_t e = hipMemcpy(tmp.data(), h->d_reps, tmp.size() * sizeof(SwRep), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading replica descriptors");
    for (size_t i = 0; i < tmp.size(); ++i) {
        SwRep& m = h->reps[i].h;
        m.thr = tmp[i].thr;
        m.p = tmp[i].p;
        if (!h->reps[i].dev_count_stale) {
            m.sweep = tmp[i].sweep;
            m.measured = tmp[i].measured;
        }
    }
    h->mirror_stale = false;
    return SW_OK;
}

// as sync_mirror, but a no-op (no wait) while the mirrors are current, so
// that back-to-back sweep calls keep the stream busy; a device error then
// surfaces at the next call that reads results
int refresh_mirror(sw_lattice* h)
{
    return h->mirror_stale ? sync_mirror(h) : SW_OK;
}

// write the full host mirror of replica r to its device descriptor (synchronous)
int push_desc(sw_lattice* h, int r)
{
    hipError_t e = hipMemcpyAsync(&h->d_reps[r], &h->reps[r].h, sizeof(SwRep), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "writing a replica descriptor");
    h->reps[r].dev_count_stale = false;
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return SW_OK;
}

// grow a device buffer of `elem`-byte entries from old_cap to new_cap, keeping contents, zeroing the rest
static int grow(void** buf, uint32_t old_cap, uint32_t new_cap, size_t elem, hipStream_t stream, const char* what)
{
    void* nb = nullptr;
    int rc = dmalloc(&nb, (size_t)new_cap * elem, what);
    if (rc) return rc;
    if (hipMemsetAsync(nb, 0, (size_t)new_cap * elem, stream) != hipSuccess ||
        (old_cap && hipMemcpyAsync(nb, *buf, (size_t)old_cap * elem, hipMemcpyDeviceToDevice, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
        dfree(nb);
        return fail(SW_EHIP, "growing the %s buffer failed", what);
    }
    dfree(*buf);
    *buf = nb;
    return SW_OK;
}

// make the series / PCC traces hold the records up to sweep `upto` (exclusive);
// records start at the replica's resume point m.first
int ensure_capacity(sw_lattice* h, int r, uint64_t upto)
{
    SwRep& m = h->reps[r].h;
    if (upto > 0xFFFFFFF0ull) return fail(SW_EINVAL, "sweep index overflow");
    const uint64_t need = upto > m.first ? upto - m.first : 0;
    bool changed = false;
    if ((m.flags & FLAG_SERIES) && need > m.series_cap) {
        int rc = refresh_mirror(h);
        if (rc) return rc;
        const uint32_t nc = (uint32_t)std::max<uint64_t>(need, 2ull * m.series_cap);
        rc = grow((void**)&m.series, m.series_cap, nc, 16, h->stream, "series");
        if (rc) return rc;
        m.series_cap = nc;
        changed = true;
    }
    if ((m.flags & FLAG_PCC) && need > m.trace_cap) {
        int rc = refresh_mirror(h);
        if (rc) return rc;
        const uint32_t nc = (uint32_t)std::max<uint64_t>(need, 2ull * m.trace_cap);
        rc = grow((void**)&m.perc_trace, m.trace_cap, nc, 4, h->stream, "percolation trace");
        if (!rc) rc = grow((void**)&m.p_trace, m.trace_cap, nc, 8, h->stream, "p trace");
        if (rc) return rc;
        m.trace_cap = nc;
        changed = true;
    }
    if (changed) return push_desc(h, r);
    return SW_OK;
}

// ---------------------------------------------------------------------------
// Per-phase timing with HIP events.
// ---------------------------------------------------------------------------
static hipEvent_t take_event(sw_lattice* h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timing_begin(sw_lattice* h, int phase, hipEvent_t* a)
{
    *a = nullptr;
    if (!h->timing) return;
    *a = take_event(h);
    if (*a) hipEventRecord(*a, h->stream);
    (void)phase;
}

void timing_end(sw_lattice* h, int phase, hipEvent_t a)
{
    if (!h->timing || !a) return;
    hipEvent_t b = take_event(h);
    if (!b) return;
    hipEventRecord(b, h->stream);
    h->pending.push_back(TimedLaunch{phase, a, b});
}

int timing_collect(sw_lattice* h)
{
    if (h->pending.empty()) return SW_OK;
    int rc = handle_sync(h);
    if (rc) return rc;
    for (auto& t : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            h->ms[t.phase] += ms;
            h->launches[t.phase] += 1;
        }
        h->event_pool.push_back(t.a);
        h->event_pool.push_back(t.b);
    }
    h->pending.clear();
    return SW_OK;
}

#define TIMED(h, phase, expr)                 \
    do {                                      \
        hipEvent_t ev_a_;                     \
        timing_begin((h), (phase), &ev_a_);   \
        int rc_ = (expr);                     \
        timing_end((h), (phase), ev_a_);      \
        if (rc_) return fail(SW_EHIP, "kernel launch failed (phase %d)", (phase)); \
    } while (0)

// ---------------------------------------------------------------------------
// Sweeps.
// ---------------------------------------------------------------------------
int plain_sweep(sw_lattice* h, int r, int32_t n)
{
    int rc = refresh_mirror(h);
    if (rc) return rc;
    ReplicaH& rep = h->reps[r];
    SwRep& m = rep.h;
    rc = ensure_capacity(h, r, (uint64_t)m.sweep + (uint64_t)n);
    if (rc) return rc;
    SwRep* d = &h->d_reps[r];
    const bool series = (m.flags & FLAG_SERIES) != 0;
    const bool pcc = (m.flags & FLAG_PCC) != 0;
    for (int32_t k = 0; k < n; ++k) {
        const uint32_t s = m.sweep + (uint32_t)k;
        int64_t* em = nullptr;
        if (series && s >= 1 && m.measured < s) {
            em = m.series + 2 * (size_t)(s - 1 - m.first);   // measured >= first, so s - 1 >= first
            m.measured = s;
        }
        TIMED(h, 0, launch_k1(m, d, s, em, h->stream, h->per_cu[0]));
        TIMED(h, 1, launch_k2(m, d, h->stream, h->merge_width));
        if (pcc && !(m.flags & FLAG_WIND)) TIMED(h, 3, launch_cand(m, d, s, h->stream));
        TIMED(h, 6, launch_k3a(m, d, s, h->stream));
        TIMED(h, 2, launch_k3(m, d, s, h->stream, h->per_cu[2]));
        if (pcc) TIMED(h, 3, launch_perc(m, d, s, h->stream));
    }
    if (pcc && n > 0) h->mirror_stale = true;   // p and thr now change on the device
    m.sweep += (uint32_t)n;
    if (series && n > 0 && m.measured < m.sweep) {
        TIMED(h, 4, launch_measure(m, d, m.series + 2 * (size_t)(m.sweep - 1 - m.first), h->stream));
        m.measured = m.sweep;
    }
    if (n > 0) {
        // the kernels of plain sweeps take the sweep index as an argument; the
        // device copy of the counters is brought up to date before a batched
        // sweep reads it
        rep.dev_count_stale = true;
        rep.labels_valid = true;
    }
    return SW_OK;
}

// The batch's groups: a mixed batch has its 2D replicas in one group and its
// 3D ones in the other; a batch of one dimension with enough tiles to fill
// the device twice over is split into two halves of about equal sites (the
// largest replica first, each to the lighter half); a small one is one group.
// The work lists hold group 0's entries, then group 1's.
static int build_items(sw_lattice* h)
{
    std::vector<int> grp(h->reps.size(), -1);
    bool has2 = false, has3 = false;
    int64_t tiles = 0;
    for (size_t r = 0; r < h->reps.size(); ++r) {
        const SwRep& m = h->reps[r].h;
        if (!m.active) continue;
        has2 = has2 || m.dim == 2;
        has3 = has3 || m.dim == 3;
        tiles += m.ntiles;
    }
    int ngroups = 1;
    if (has2 && has3) {
        ngroups = 2;
        for (size_t r = 0; r < h->reps.size(); ++r)
            if (h->reps[r].h.active) grp[r] = h->reps[r].h.dim == 2 ? 0 : 1;
    } else {
        std::vector<int> order;
        for (size_t r = 0; r < h->reps.size(); ++r)
            if (h->reps[r].h.active) order.push_back((int)r);
        ngroups = (order.size() >= 2 && tiles >= 4 * (int64_t)device_cu_count()) ? 2 : 1;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return h->reps[x].h.N > h->reps[y].h.N; });
        uint64_t load[2] = {0, 0};
        for (int r : order) {
            const int g = (ngroups == 2 && load[1] < load[0]) ? 1 : 0;
            grp[r] = g;
            load[g] += h->reps[r].h.N;
        }
    }
    std::vector<EngineItem> items, cand, perc, reps;
    for (int g = 0; g < ngroups; ++g) {
        BatchGroup& G = h->groups[g];
        G.item0 = (int)items.size();
        G.cand0 = (int)cand.size();
        G.perc0 = (int)perc.size();
        G.rep0 = (int)reps.size();
        G.dim = 0;
        for (size_t r = 0; r < h->reps.size(); ++r) {
            if (grp[r] != g) continue;
            const SwRep& m = h->reps[r].h;
            G.dim = m.dim;
            reps.push_back(EngineItem{(int32_t)r, 0});
            for (int t = 0; t < m.ntiles; ++t) {
                items.push_back(EngineItem{(int32_t)r, t});
                const int ix = t % m.ntx, iy = (t / m.ntx) % m.nty, iz = t / (m.ntx * m.nty);
                if ((m.flags & (FLAG_PCC | FLAG_WIND)) == FLAG_PCC && (ix == 0 || iy == 0 || (m.dim == 3 && iz == 0)))
                    cand.push_back(EngineItem{(int32_t)r, t});
            }
            if ((m.flags & (FLAG_PCC | FLAG_WIND)) == FLAG_PCC) {
                const int64_t nslots = (m.dim == 3) ? (int64_t)m.L * m.L : (int64_t)m.L;
                for (int64_t k = 0; k * kPercChunk < nslots; ++k) perc.push_back(EngineItem{(int32_t)r, (int32_t)k});
            }
        }
        G.nitems = (int)items.size() - G.item0;
        G.ncand = (int)cand.size() - G.cand0;
        G.nperc = (int)perc.size() - G.perc0;
        G.nrep = (int)reps.size() - G.rep0;
    }
    h->ngroups = ngroups;
    const size_t nlist = items.size();
    h->ncand = (int)cand.size();
    h->nperc = (int)perc.size();
    h->nreplist = (int)reps.size();
    items.insert(items.end(), cand.begin(), cand.end());
    items.insert(items.end(), perc.begin(), perc.end());
    items.insert(items.end(), reps.begin(), reps.end());
    if (h->items_cap < items.size()) {
        dfree(h->items);
        h->items = nullptr;
        h->items_cap = 0;
        int rc = dmalloc((void**)&h->items, std::max<size_t>(items.size(), 1) * sizeof(EngineItem), "engine work list");
        if (rc) return rc;
        h->items_cap = items.size();
    }
    if (!items.empty()) {
        hipError_t e = hipMemcpy(h->items, items.data(), items.size() * sizeof(EngineItem), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "uploading the engine work list");
    }
    if (ngroups == 2 && !h->side) {
        hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "creating the second batch stream");
    }
    h->nitems = (int)nlist;
    h->items_dirty = false;
    h->graph_n = -1;    // work list changed: re-capture
    return SW_OK;
}

static void drop_graph(sw_lattice* h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->graph_n = -1;
}

// the batched kernels are compiled for pairs (2D shape i, 3D shape i): all
// active replicas of a batched handle must use the same shape index
int engine_variant(sw_lattice* h, int* variant)
{
    int v = -1;
    for (auto& r : h->reps) {
        if (!r.h.active) continue;
        if (v < 0) v = r.h.shape;
        else if (r.h.shape != v)
            return fail(SW_ESTATE, "batched mode needs every replica on the same tile-shape index (%d and %d)", v,
                        r.h.shape);
    }
    *variant = v < 0 ? 0 : v;
    return SW_OK;
}

int batched_sweep(sw_lattice* h, int32_t n)
{
    int rc = refresh_mirror(h);
    if (rc) return rc;
    for (auto& rep : h->reps) {
        if (!rep.dev_count_stale) continue;
        const SwRep& m = rep.h;
        if (launch_set_state(&h->d_reps[&rep - h->reps.data()], m.sweep, m.measured, m.first, 0.0, 0, 0, h->stream))
            return fail(SW_EHIP, "state update launch failed");
        rep.dev_count_stale = false;
    }
    int pcc_dims = 0;   // bit 0: a 2D PCC replica is active, bit 1: a 3D one
    bool any_series = false, any_3d = false, any_2d = false;
    for (size_t r = 0; r < h->reps.size(); ++r) {
        SwRep& m = h->reps[r].h;
        if (!m.active) continue;
        rc = ensure_capacity(h, (int)r, std::min<uint64_t>((uint64_t)m.sweep + (uint64_t)n, (uint64_t)m.limit));
        if (rc) return rc;
        if (m.flags & FLAG_PCC) pcc_dims |= (m.dim == 2) ? 1 : 2;
        any_series = any_series || (m.flags & FLAG_SERIES);
        any_3d = any_3d || m.dim == 3;
        any_2d = any_2d || m.dim == 2;
    }
    if (h->items_dirty || !h->items) {
        rc = build_items(h);
        if (rc) return rc;
    }
    if (h->nitems == 0 || n == 0) return SW_OK;
    int variant = 0;
    rc = engine_variant(h, &variant);
    if (rc) return rc;
    // list-chunking kernels: per_cu workgroups per CU (8 when the phase
    // kernels take one workgroup per tile); phase kernels: one workgroup per
    // tile, or per_cu per CU each running a chunk of the list
    auto clamp_grid = [&](int g) {
        g = std::min(g, h->nitems);
        if (g >= 8) g -= g % 8;
        return g < 1 ? 1 : g;
    };
    const int per_cu = h->batch_per_cu;
    if (h->batch_engine == SW_ENGINE_PERSISTENT) {
        hipEvent_t ev;
        timing_begin(h, 5, &ev);
        int lrc = launch_persistent(variant, h->d_reps, (int)h->reps.size(), h->items, h->nitems, h->items + h->nitems,
                                    h->ncand, h->items + h->nitems + h->ncand, h->nperc, n, pcc_dims, any_series,
                                    (int)any_2d | ((int)any_3d << 1), per_cu, h->bar, h->err, h->stream,
                                    &h->persist_grid);
        timing_end(h, 5, ev);
        if (lrc) return fail(SW_EHIP, "persistent batched launch failed (%d)", lrc);
        h->mirror_stale = true;
        for (auto& rep : h->reps)
            if (rep.h.active) rep.labels_valid = true;
        return SW_OK;
    }
    const int grid = clamp_grid(device_cu_count() * (per_cu > 0 ? per_cu : 8));
    const int item_grid = per_cu > 0 ? clamp_grid(device_cu_count() * per_cu) : h->nitems;
    if (h->graph_n != n || h->graph_grid != grid || h->graph_item_grid != item_grid || h->graph_merge != h->merge_width ||
        h->graph_flags != (int)(any_2d * 16 + any_3d * 8 + pcc_dims * 2 + any_series) || h->graph_variant != variant) {
        drop_graph(h);
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const EngineItem* cand = h->items + h->nitems;
        int lrc = launch_batch(variant, h->d_reps, (int)h->reps.size(), h->items, h->nitems, cand, cand + h->ncand,
                               cand + h->ncand + h->nperc, h->groups, h->ngroups, n, pcc_dims, any_series, grid,
                               item_grid, h->merge_width, h->stream, h->side, h->fork_ev, h->join_ev);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->stream, &g);
        if (lrc || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(SW_EHIP, "capturing the batched launches failed");
        }
        h->graph = g;
        e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(h);
            return hip_fail(e, "hipGraphInstantiate");
        }
        h->graph_n = n;
        h->graph_grid = grid;
        h->graph_item_grid = item_grid;
        h->graph_merge = h->merge_width;
        h->graph_flags = (int)(any_2d * 16 + any_3d * 8 + pcc_dims * 2 + any_series);
        h->graph_variant = variant;
    }
    hipEvent_t ev;
    timing_begin(h, 5, &ev);
    hipError_t e = hipGraphLaunch(h->gexec, h->stream);
    timing_end(h, 5, ev);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    h->mirror_stale = true;
    for (auto& rep : h->reps)
        if (rep.h.active) rep.labels_valid = true;
    return SW_OK;
}

}  // namespace sw

using namespace sw;

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
extern "C" {

void sw_params_default(sw_params* p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->dim = 2;
    p->L = 64;
    p->J = 1.0;
    p->T = 2.0 / std::log(1.0 + std::sqrt(2.0));
    p->p_bond = -1.0;
    p->seed = 1;
    p->flags = 0;
    p->pcc_dp0 = 0.01;
    p->pcc_halve_every = 1000;
    p->series_cap = 0;
}

const char* sw_last_error(void) { return last_error(); }

int sw_init(const sw_params* params, int32_t n_replicas, int32_t device, void* hip_stream, sw_lattice** out)
{
    if (!out) return fail(SW_EINVAL, "null output handle");
    if (!params || n_replicas < 1) return fail(SW_EINVAL, "need at least one replica");
    for (int32_t r = 0; r < n_replicas; ++r) {
        int rc = validate_params(&params[r]);
        if (rc) return rc;
    }
    int dev = device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return fail(SW_EHIP, "no HIP device");
    }
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    sw_lattice* h = new (std::nothrow) sw_lattice();
    if (!h) return fail(SW_ENOMEM, "host allocation failed");
    h->device = dev;
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
        h->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "hipStreamCreate");
        }
        h->own_stream = true;
    }
    h->reps.resize(n_replicas);
    int rc = SW_OK;
    for (int32_t r = 0; r < n_replicas && !rc; ++r) rc = replica_alloc(h->reps[r], &params[r], default_shape(params[r].dim), h->stream);
    if (!rc) rc = dmalloc((void**)&h->d_reps, sizeof(SwRep) * (size_t)n_replicas, "replica descriptors");
    // the error word, and 128 bytes further the persistent engine's barrier word
    if (!rc) rc = dmalloc((void**)&h->err, 256, "consistency-check and barrier words");
    if (!rc && hipMemsetAsync(h->err, 0, 256, h->stream) != hipSuccess)
        rc = fail(SW_EHIP, "clearing the consistency-check word");
    if (!rc) h->bar = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(h->err) + 128);
    if (!rc) {
        std::vector<SwRep> tmp(n_replicas);
        for (int32_t r = 0; r < n_replicas; ++r) {
            h->reps[r].h.err = h->err;
            tmp[r] = h->reps[r].h;
        }
        e = hipMemcpyAsync(h->d_reps, tmp.data(), tmp.size() * sizeof(SwRep), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) rc = hip_fail(e, "uploading replica descriptors");
        if (!rc) e = hipStreamSynchronize(h->stream);
        if (!rc && e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    for (int32_t r = 0; r < n_replicas && !rc; ++r)
        if (launch_init(h->reps[r].h, &h->d_reps[r], h->stream)) rc = fail(SW_EHIP, "init kernel launch failed");
    if (!rc) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = hip_fail(e, "initial spins");
    }
    if (rc) {
        sw_free(h);
        return rc;
    }
    *out = h;
    return SW_OK;
}

int sw_set_mode(sw_lattice* h, int32_t mode)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (mode != SW_MODE_PLAIN && mode != SW_MODE_BATCHED) return fail(SW_EINVAL, "unknown mode %d", mode);
    h->mode = mode;
    return SW_OK;
}

int sw_set_batch_grid(sw_lattice* h, int32_t per_cu)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (per_cu < 0 || per_cu > 64) return fail(SW_EINVAL, "workgroups per CU must be in [0, 64] (got %d)", per_cu);
    h->batch_per_cu = per_cu;
    return SW_OK;
}

int sw_get_batch_grid(sw_lattice* h, int32_t* per_cu)
{
    if (!h || !per_cu) return fail(SW_EINVAL, "null argument");
    *per_cu = h->batch_per_cu;
    return SW_OK;
}

int sw_set_batch_engine(sw_lattice* h, int32_t engine)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (engine != SW_ENGINE_GRAPH && engine != SW_ENGINE_PERSISTENT)
        return fail(SW_EINVAL, "unknown batched engine %d", engine);
    h->batch_engine = engine;
    return SW_OK;
}

int sw_get_batch_engine(sw_lattice* h, int32_t* engine, int32_t* grid)
{
    if (!h || !engine) return fail(SW_EINVAL, "null argument");
    *engine = h->batch_engine;
    if (grid) *grid = h->persist_grid;
    return SW_OK;
}

int sw_set_merge_width(sw_lattice* h, int32_t threads)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (threads != 0 && threads != 64 && threads != 256)
        return fail(SW_EINVAL, "border-merge width must be 0, 64 or 256 (got %d)", threads);
    h->merge_width = threads;
    return SW_OK;
}

int sw_get_merge_width(sw_lattice* h, int32_t* threads)
{
    if (!h || !threads) return fail(SW_EINVAL, "null argument");
    *threads = h->merge_width;
    return SW_OK;
}

int sw_sweep(sw_lattice* h, int32_t n_sweeps)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    if (n_sweeps < 0) return fail(SW_EINVAL, "negative sweep count");
    int rc = set_device(h);
    if (rc) return rc;
    if (h->mode == SW_MODE_BATCHED) return batched_sweep(h, n_sweeps);
    for (size_t r = 0; r < h->reps.size(); ++r) {
        rc = plain_sweep(h, (int)r, n_sweeps);
        if (rc) return rc;
    }
    return SW_OK;
}

int sw_sweep_replica(sw_lattice* h, int32_t replica, int32_t n_sweeps)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(SW_EINVAL, "negative sweep count");
    rc = set_device(h);
    if (rc) return rc;
    return plain_sweep(h, replica, n_sweeps);
}

int sw_measure(sw_lattice* h, int32_t replica, int64_t* e_int, int64_t* m)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    if (!e_int || !m) return fail(SW_EINVAL, "null output");
    rc = set_device(h);
    if (rc) return rc;
    SwRep& mm = h->reps[replica].h;
    if (hipMemsetAsync(mm.acc, 0, 16, h->stream) != hipSuccess) return fail(SW_EHIP, "clearing accumulators");
    TIMED(h, 4, launch_measure(mm, &h->d_reps[replica], mm.acc, h->stream));
    int64_t v[2];
    hipError_t e = hipMemcpyAsync(v, mm.acc, 16, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "reading accumulators");
    rc = handle_sync(h);
    if (rc) return rc;
    *e_int = v[0];
    *m = v[1];
    return SW_OK;
}

int sw_get_series(sw_lattice* h, int32_t replica, int64_t* host_buf, int64_t cap, int64_t* count,
                  int64_t* first_sweep)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    SwRep& m = h->reps[replica].h;
    if (!(m.flags & FLAG_SERIES)) return fail(SW_ESTATE, "replica does not record a series");
    if (!host_buf || !count || cap < 0) return fail(SW_EINVAL, "bad output buffer");
    rc = set_device(h);
    if (!rc) rc = sync_mirror(h);
    if (rc) return rc;
    // rows of the sweeps [first, measured): never more than the buffer holds
    const int64_t have = m.measured > m.first ? (int64_t)(m.measured - m.first) : 0;
    const int64_t nrec = std::min<int64_t>(std::min<int64_t>(have, (int64_t)m.series_cap), cap / 2);
    if (nrec > 0) {
        hipError_t e = hipMemcpy(host_buf, m.series, (size_t)nrec * 16, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the series");
    }
    *count = nrec;
    if (first_sweep) *first_sweep = m.first;
    return SW_OK;
}

int sw_get_spins(sw_lattice* h, int32_t replica, int8_t* host_buf, int64_t cap)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    SwRep& m = h->reps[replica].h;
    if (!host_buf || cap < (int64_t)m.N) return fail(SW_EINVAL, "buffer smaller than N");
    rc = set_device(h);
    if (!rc) rc = handle_sync(h);
    if (rc) return rc;
    return read_spins(m, host_buf);
}

int sw_get_labels(sw_lattice* h, int32_t replica, int32_t* host_buf, int64_t cap)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    SwRep& m = h->reps[replica].h;
    if (!m.lab32) return fail(SW_ESTATE, "labels are kept only with SW_KEEP_LABELS");
    if (!h->reps[replica].labels_valid) return fail(SW_ESTATE, "no sweep done yet");
    if (!host_buf || cap < (int64_t)m.N) return fail(SW_EINVAL, "buffer smaller than N");
    rc = set_device(h);
    if (!rc) rc = handle_sync(h);
    if (rc) return rc;
    hipError_t e = hipMemcpy(host_buf, m.lab32, (size_t)m.N * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? SW_OK : hip_fail(e, "reading labels");
}

int sw_get_state(sw_lattice* h, int32_t replica, uint32_t* sweep, double* p, uint64_t* thr)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    rc = set_device(h);
    if (rc) return rc;
    h->mirror_stale = true;
    rc = sync_mirror(h);
    if (rc) return rc;
    const SwRep& m = h->reps[replica].h;
    if (sweep) *sweep = m.sweep;
    if (p) *p = m.p;
    if (thr) *thr = m.thr;
    return SW_OK;
}

int sw_get_pcc_trace(sw_lattice* h, int32_t replica, int32_t* perc, double* p, int64_t cap, int64_t* count,
                     int64_t* first_sweep)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    SwRep& m = h->reps[replica].h;
    if (!(m.flags & FLAG_PCC)) return fail(SW_ESTATE, "replica is not a PCC replica");
    if (!count || cap < 0) return fail(SW_EINVAL, "bad output");
    rc = set_device(h);
    if (!rc) rc = sync_mirror(h);
    if (rc) return rc;
    const int64_t have = m.sweep > m.first ? (int64_t)(m.sweep - m.first) : 0;
    const int64_t n = std::min<int64_t>(std::min<int64_t>(have, (int64_t)m.trace_cap), cap);
    if (n > 0 && perc) {
        hipError_t e = hipMemcpy(perc, m.perc_trace, (size_t)n * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the percolation trace");
    }
    if (n > 0 && p) {
        hipError_t e = hipMemcpy(p, m.p_trace, (size_t)n * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the p trace");
    }
    *count = n;
    if (first_sweep) *first_sweep = m.first;
    return SW_OK;
}

int sw_set_spins(sw_lattice* h, int32_t replica, const int8_t* host_buf, int64_t n, uint32_t sweep, double p)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    SwRep& m = h->reps[replica].h;
    if (!host_buf || n != (int64_t)m.N) return fail(SW_EINVAL, "need exactly N spins");
    for (int64_t i = 0; i < n; ++i)
        if (host_buf[i] != 1 && host_buf[i] != -1) return fail(SW_EINVAL, "spin %lld is not +1/-1", (long long)i);
    const bool pcc = (m.flags & FLAG_PCC) != 0;
    if (pcc && !(p >= 0.0 && p <= 1.0)) return fail(SW_EINVAL, "p must be in [0,1]");
    if (sweep > 0xFFFFFFF0u) return fail(SW_EINVAL, "sweep index too large");
    rc = set_device(h);
    if (!rc) rc = sync_mirror(h);
    if (rc) return rc;
    rc = write_spins(m, host_buf);
    if (rc) return rc;
    // The records restart at the resume point.  Series rows are accumulated
    // with atomic adds, so the reused rows are cleared; PCC candidate marks
    // carry the tag of the sweep that wrote them, and a tag left by a later
    // sweep of the abandoned trajectory would outrank this one's, so they are
    // cleared too (with the coverage bitmaps and the flag, which are zero
    // between sweeps anyway).
    m.sweep = sweep;
    m.measured = sweep;
    m.first = sweep;
    if ((m.flags & FLAG_SERIES) && hipMemsetAsync(m.series, 0, (size_t)m.series_cap * 16, h->stream) != hipSuccess)
        return fail(SW_EHIP, "clearing the series failed");
    if (pcc) {
        m.p = p;
        m.thr = threshold_from_p(p);
        const size_t L = (size_t)m.L;
        const size_t ns = (m.dim == 3) ? L * L : L;
        if (hipMemsetAsync(m.cand, 0, (size_t)m.dim * m.N * 8, h->stream) != hipSuccess ||
            hipMemsetAsync(m.bmp, 0, (size_t)m.dim * ns * ((L + 31) / 32) * 4, h->stream) != hipSuccess ||
            hipMemsetAsync(m.pflag, 0, 16, h->stream) != hipSuccess)
            return fail(SW_EHIP, "clearing the percolation buffers failed");
    }
    h->reps[replica].labels_valid = false;
    if (launch_set_state(&h->d_reps[replica], m.sweep, m.measured, m.first, m.p, m.thr, pcc ? 1 : 0, h->stream))
        return fail(SW_EHIP, "state update launch failed");
    h->reps[replica].dev_count_stale = false;
    return handle_sync(h);
}

int sw_bind_device_spins(sw_lattice* h, int32_t replica, void* dev_ptr)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    if (!dev_ptr) return fail(SW_EINVAL, "null device pointer");
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 15u)
        return fail(SW_EINVAL, "the spin array must be 16-byte aligned (the kernels move whole vectors of spins)");
    rc = set_device(h);
    if (!rc) rc = sync_mirror(h);
    if (rc) return rc;
    ReplicaH& r = h->reps[replica];
    if (r.own_spins) dfree(r.h.spins);
    r.h.spins = (int8_t*)dev_ptr;
    r.own_spins = false;
    return push_desc(h, replica);
}

int sw_set_timing(sw_lattice* h, int32_t enable)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    int rc = timing_collect(h);
    if (rc) return rc;
    h->timing = enable != 0;
    for (int k = 0; k < kPhases; ++k) {
        h->ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return SW_OK;
}

int sw_get_timing(sw_lattice* h, double* ms, int64_t* launches, int32_t n)
{
    if (!h) return fail(SW_EINVAL, "null handle");
    int rc = timing_collect(h);
    if (rc) return rc;
    for (int k = 0; k < n && k < kPhases; ++k) {
        if (ms) ms[k] = h->ms[k];
        if (launches) launches[k] = h->launches[k];
    }
    return SW_OK;
}

int sw_set_tile_shape(sw_lattice* h, int32_t replica, int32_t shape)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    ReplicaH& r = h->reps[replica];
    if (shape < 0 || shape >= shape_count(r.h.dim)) return fail(SW_EINVAL, "unknown tile shape %d", shape);
    rc = set_device(h);
    if (!rc) rc = sync_mirror(h);
    if (rc) return rc;
    if (shape == r.h.shape) return SW_OK;
    SwRep probe = r.h;
    fill_geometry(probe, shape);
    rc = alloc_tile_buffers(probe);
    if (rc) return rc;
    free_tile_buffers(r.h);
    r.h = probe;
    h->items_dirty = true;
    return push_desc(h, replica);
}

int sw_get_tile_shape(sw_lattice* h, int32_t replica, int32_t* shape)
{
    int rc = check_rep(h, replica);
    if (rc) return rc;
    if (!shape) return fail(SW_EINVAL, "null output");
    *shape = h->reps[replica].h.shape;
    return SW_OK;
}

int sw_tile_shapes(int32_t dim, int32_t* count, int32_t* tx, int32_t* ty, int32_t* tz, int32_t cap)
{
    if (dim != 2 && dim != 3) return fail(SW_EINVAL, "dim must be 2 or 3");
    const int n = shape_count(dim);
    if (count) *count = n;
    for (int i = 0; i < n && i < cap; ++i) {
        int a, b, c;
        shape_extents(dim, i, &a, &b, &c);
        if (tx) tx[i] = a;
        if (ty) ty[i] = b;
        if (tz) tz[i] = c;
    }
    return SW_OK;
}

int sw_free(sw_lattice* h)
{
    if (!h) return SW_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& t : h->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    drop_graph(h);
    for (auto& r : h->reps) replica_free(r);
    dfree(h->d_reps);
    dfree(h->items);
    dfree(h->err);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return SW_OK;
}

}  // extern "C"
