/*
 * sw_api.h -- C ABI of libswgpu.so, the MI355X (gfx950) Swendsen-Wang sweep
 * engine for the Ising model H = -J sum_<ij> s_i s_j.
 *
 * One sweep is the cluster update of Lin & Zheng, Sec. I, steps 1-3:
 *   1. every link between equal neighbours becomes a bond with probability
 *      P = 1 - exp(-2J/T);
 *   2. sites joined by a path of bonds form a cluster;
 *   3. every cluster takes one fresh random spin, shared by all its sites.
 * On top of the plain sweep the library runs the probability-changing-cluster
 * feedback of Sec. III (extension rule, periodic boundaries), many replicas
 * swept together by one hipGraph launch, and a continuous-batching job server.
 *
 * Conventions shared by every entry point
 *   - Lattices are periodic (open with SW_OPEN), dim 2 or 3, N = L^dim sites, site index
 *     i = x + L*y (+ L*L*z), x fastest.  Link (i,d) joins i and i + e_d.
 *   - Spins are int8 +1/-1.  Labels are int32: the canonical label of a
 *     cluster is the smallest site index it contains.
 *   - Random stream SWRNG-1 (the paper names none): Philox4x32-10 keyed by the
 *     64-bit seed, counter (block, 0, sweep, tag).  Initial spin of site i: bit
 *     i%32 of word (i>>5)%4 of block i>>7 (tag 0).  Bond of link l = d*N + i:
 *     u = a*2^24 + b with a = byte l%16 of block l>>4 (tag 1) and b = low 24
 *     bits of word l%4 of block l>>2 (tag 2); the link opens when the spins are
 *     equal and u < thr, thr = min(2^32, floor(P * 2^32)).  New spin of the
 *     cluster labelled r: bit r%32 of word (r>>5)%4 of block r>>7 (tag 3).
 *     A trajectory is therefore a pure function of (parameters, seed) and is
 *     reproduced bit for bit by any schedule, tile shape or batch mix.
 *   - Every function returns an int status: SW_OK (0) or a negative SW_E*
 *     code; sw_last_error() then describes the failure.  No C++ exception
 *     crosses the boundary.  Output arguments are written only on SW_OK.
 *   - Ownership: a handle owns the device memory it allocates and frees it in
 *     sw_free / sw_server_destroy.  Host buffers always belong to the caller.
 *     A device buffer bound with sw_bind_device_spins stays the caller's.
 *   - Streams: `hip_stream` is a hipStream_t passed as void* (NULL: the handle
 *     creates and owns a stream).  Sweeps are enqueued asynchronously; every
 *     sw_get_* / sw_measure call synchronises the handle's stream and checks
 *     the device consistency word, so a failure detected on the device during
 *     sweeps is returned (SW_EHIP) by the next such call.
 *   - Handles are not thread-safe; a server serialises its own calls.
 */
#ifndef SW_API_H
#define SW_API_H

#include <stdint.h>

#if defined(SW_BUILD_LIBRARY) && defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SW_OK = 0,
    SW_EINVAL = -1,      /* invalid argument or parameter set            */
    SW_ENOMEM = -2,      /* device or host allocation failed             */
    SW_EHIP = -3,        /* a HIP runtime call or kernel launch failed   */
    SW_EBUSY = -4,       /* resource in use (server slot table full, ...) */
    SW_ENOTFOUND = -5,   /* unknown job id                               */
    SW_ECANCELLED = -6,  /* job was cancelled                            */
    SW_ESTATE = -7       /* call not valid in the object's current state */
};

/* flags of sw_params.flags */
enum {
    SW_RECORD_SERIES = 1u << 0, /* record (E_int, M) after every sweep          */
    SW_KEEP_LABELS = 1u << 1,   /* keep the int32 labels of the last sweep       */
    SW_PCC = 1u << 2,           /* probability-changing-cluster feedback (Sec. III) */
    SW_BITPACK = 1u << 3,       /* keep the spins (the +-1 of Sec. I) as one bit per
                                   site on the device: ceil(N/32) uint32 words, site
                                   i up iff bit i%32 of word i/32 is set.  Every
                                   result is the same as with int8 spins; sw_get_spins
                                   and sw_set_spins still take int8 arrays. */
    SW_OPEN = 1u << 4,          /* open boundaries in every axis (Sec. III discusses
                                   both kinds): the links that would wrap around the
                                   box do not exist (every other link keeps its index
                                   and draw), E_int sums over the box's links, and the
                                   PCC test is the open box's spanning test: one
                                   cluster holds sites of both opposite faces
                                   (coordinate 0 and L-1) of some axis. */
    SW_PCC_WIND = 1u << 5       /* with SW_PCC on a periodic box: percolation by the
                                   topological rule of Sec. III (one cluster winds
                                   around the box along some axis) instead of the
                                   extension rule; SW_EINVAL without SW_PCC or with
                                   SW_OPEN */
};

/* execution modes of a multi-replica handle (sw_set_mode) */
enum {
    SW_MODE_PLAIN = 0,    /* one launch sequence per replica and sweep            */
    SW_MODE_BATCHED = 1   /* all replicas' tiles in each phase launch, the sweeps
                             of one call replayed as one hipGraph                 */
};

/*
 * Parameters of one lattice (replica).
 *   dim             2 or 3
 *   L               linear size, >= 3, with L^dim < 2^31 and dim*L^dim < 2^32
 *   J, T            coupling (> 0, ferromagnet as in Sec. I) and temperature (> 0)
 *   p_bond          < 0: P = 1 - exp(-2J/T) (evaluated as -expm1(-2J/T) in double);
 *                   in [0,1]: use this P directly (the PCC start value)
 *   seed            key of the random stream
 *   flags           SW_RECORD_SERIES | SW_KEEP_LABELS | SW_PCC | SW_BITPACK | SW_OPEN | SW_PCC_WIND
 *   pcc_dp0         PCC step dp at sweep 0 (> 0)
 *   pcc_halve_every dp is halved every this many sweeps (> 0)
 *   series_cap      capacity of the (E_int, M) series in sweeps (0: grows on demand)
 */
typedef struct sw_params {
    int32_t dim;
    int32_t L;
    double J;
    double T;
    double p_bond;
    uint64_t seed;
    uint32_t flags;
    double pcc_dp0;
    uint32_t pcc_halve_every;
    uint32_t series_cap;
} sw_params;

/* Fill *p with defaults: dim 2, L 64, J 1, T = 2/ln(1+sqrt 2), p_bond -1, seed 1,
 * flags 0, pcc_dp0 0.01, pcc_halve_every 1000, series_cap 0. */
void sw_params_default(sw_params* p);

/* ------------------------------------------------------------------------ */
/* Lattices                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct sw_lattice sw_lattice;

/*
 * Create a handle holding n_replicas independent lattices; params[r] describes
 * replica r (replicas may differ in dim, L, T, seed and flags).  Spins start
 * from the SWRNG-1 initial draw.  All parameters are validated before any
 * allocation (SW_EINVAL).  `device` selects the HIP device (-1: current).
 */
int sw_init(const sw_params* params, int32_t n_replicas, int32_t device, void* hip_stream,
            sw_lattice** out);

/* Choose how sw_sweep runs the replicas (SW_MODE_PLAIN or SW_MODE_BATCHED). */
int sw_set_mode(sw_lattice* h, int32_t mode);

/* Launch shape of batched sweeps: per_cu = 0 runs the per-tile phases with one
 * workgroup per tile of every active replica; per_cu in [1, 64] runs them with
 * per_cu workgroups per compute unit, each taking a contiguous chunk of the
 * (replica, tile) list.  Results never depend on it (every union hooks to the
 * smaller root, so the schedule cannot change a label); the autotuner sets it
 * too.  SW_EINVAL outside [0, 64]. */
int sw_set_batch_grid(sw_lattice* h, int32_t per_cu);

/* Current launch shape of batched sweeps (see sw_set_batch_grid). */
int sw_get_batch_grid(sw_lattice* h, int32_t* per_cu);

/* Batched engines (sw_set_batch_engine). */
enum {
    SW_ENGINE_GRAPH = 0,       /* one kernel per phase, n sweeps captured in a replayed hipGraph (default) */
    SW_ENGINE_PERSISTENT = 1   /* one cooperative launch per call (per 4096 sweeps): resident workgroups walk
                                  the phases with a software grid barrier between them */
};

/* Choose how batched sweeps run (Sec. II's sweep for many replicas at once):
 * both engines run the same per-tile work in the same order of phases and give
 * identical results.  The persistent engine sizes its grid to the workgroups
 * that fit on the device at once (or sw_set_batch_grid's per-CU count, if
 * smaller) and always uses 256-thread border merges.  A barrier that waits
 * more than 10 s abandons the launch and sets a consistency error, which the
 * next synchronising call reports as SW_EHIP.  SW_EINVAL for unknown engines. */
int sw_set_batch_engine(sw_lattice* h, int32_t engine);

/* Current batched engine; grid (may be NULL) receives the workgroups of the
 * last persistent launch (0 before the first). */
int sw_get_batch_engine(sw_lattice* h, int32_t* engine, int32_t* grid);

/* Merge schedule of the border merge (the global union across tile faces that
 * reconciles the domains' labels, Sec. II): threads per tile, 64 (one wave per
 * tile: more tiles in flight) or 256 (each thread fewer face sites); 0 picks
 * per tile shape.  Results never depend on it; the autotuner sets it too.
 * SW_EINVAL for other values. */
int sw_set_merge_width(sw_lattice* h, int32_t threads);

/* Current merge schedule (see sw_set_merge_width). */
int sw_get_merge_width(sw_lattice* h, int32_t* threads);

/*
 * Advance every replica by n_sweeps sweeps (Sec. I steps 1-3, plus the PCC
 * feedback of Sec. III for SW_PCC replicas).  Asynchronous on the stream.
 */
int sw_sweep(sw_lattice* h, int32_t n_sweeps);

/* Advance only replica r by n_sweeps sweeps with plain launches. */
int sw_sweep_replica(sw_lattice* h, int32_t replica, int32_t n_sweeps);

/* E_int = sum over links of s_i s_j (H = -J E_int) and M = sum s_i of the
 * current configuration of a replica.  Synchronises. */
int sw_measure(sw_lattice* h, int32_t replica, int64_t* e_int, int64_t* m);

/* Copy the recorded (E_int, M) series of a SW_RECORD_SERIES replica into
 * host_buf (cap int64 entries, 2 per sweep): row j holds E_int and M of the
 * configuration after sweep first + j, where first is the resume point of the
 * last sw_set_spins (0 for a handle never rewound).  *count receives the
 * number of rows copied, *first_sweep (may be NULL) the value of first.  Only
 * measured rows are copied, never more than the device buffer holds.
 * Synchronises. */
int sw_get_series(sw_lattice* h, int32_t replica, int64_t* host_buf, int64_t cap, int64_t* count,
                  int64_t* first_sweep);

/* Copy the N spins of a replica to host memory as int8 +1/-1 (cap >= N; a
 * bit-packed replica is unpacked on the host).  Synchronises. */
int sw_get_spins(sw_lattice* h, int32_t replica, int8_t* host_buf, int64_t cap);

/* Copy the N canonical labels of the last sweep (needs SW_KEEP_LABELS and at
 * least one sweep done).  Synchronises. */
int sw_get_labels(sw_lattice* h, int32_t replica, int32_t* host_buf, int64_t cap);

/* Current sweep index (sweeps done), bond probability p and threshold thr of a
 * replica.  Synchronises. */
int sw_get_state(sw_lattice* h, int32_t replica, uint32_t* sweep, double* p, uint64_t* thr);

/* Copy the per-sweep percolation flags (extension rule, Sec. III) and the p
 * values after each feedback step of a SW_PCC replica: entry j belongs to
 * sweep first + j (first as in sw_get_series); count = min(cap, sweeps done
 * since first).  perc or p may be NULL.  Synchronises. */
int sw_get_pcc_trace(sw_lattice* h, int32_t replica, int32_t* perc, double* p, int64_t cap,
                     int64_t* count, int64_t* first_sweep);

/* Replace a replica's spins (N int8 of +1/-1, host memory) and set its sweep
 * index to `sweep` (checkpoint / resume), forward or back.  For SW_PCC
 * replicas p (in [0,1]) becomes the current bond probability; otherwise p is
 * ignored.  The series and PCC trace restart at `sweep` (their rows before it
 * are dropped), and every per-sweep mark left by the abandoned trajectory is
 * cleared, so the continuation equals a fresh run from this state.
 * Synchronises. */
int sw_set_spins(sw_lattice* h, int32_t replica, const int8_t* host_buf, int64_t n, uint32_t sweep,
                 double p);

/* Use a caller-owned device buffer as the replica's spin array (its contents
 * become the current configuration): N int8 of +1/-1, or for a SW_BITPACK
 * replica ceil(N/32) uint32 words in the packed layout, 16-byte aligned
 * (SW_EINVAL otherwise).  The library never frees it; it must stay valid until
 * sw_free or the next bind. */
int sw_bind_device_spins(sw_lattice* h, int32_t replica, void* dev_ptr);

/* Enable per-phase kernel timing with HIP events on the handle's stream. */
int sw_set_timing(sw_lattice* h, int32_t enable);

/*
 * Accumulated device time per phase since timing was enabled: ms[k] and
 * launches[k] for k < n (k = 0 bond+tile labelling, 1 border merge, 2 cluster
 * flip, 3 percolation + feedback, 4 measurement, 5 batched sweeps: one
 * replayed graph per call, all phases together, 6 border-root resolution).
 * Synchronises.
 */
int sw_get_timing(sw_lattice* h, double* ms, int64_t* launches, int32_t n);

/* Tile shape used for each replica (0 = autotuned default).  `shape` indexes
 * sw_tile_shapes(). */
int sw_set_tile_shape(sw_lattice* h, int32_t replica, int32_t shape);

/* Tile shape currently used by a replica (index into sw_tile_shapes()). */
int sw_get_tile_shape(sw_lattice* h, int32_t replica, int32_t* shape);

/* Number of compiled tile shapes and their extents (tx, ty, tz; tz = 1 in 2D). */
int sw_tile_shapes(int32_t dim, int32_t* count, int32_t* tx, int32_t* ty, int32_t* tz, int32_t cap);

/*
 * Autotune: for every (dim, size class) present in the handle, time each
 * compiled tile shape (and, for batches, the workgroups per CU) on scratch copies for
 * `sweeps` sweeps and keep the fastest.  Results are written to / read from
 * the JSON cache at `cache_path` (NULL: no cache).  Trajectories do not
 * depend on the choice.  Synchronises.
 */
int sw_autotune(sw_lattice* h, int32_t sweeps, const char* cache_path);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): n_sweeps
 * sweeps of one lattice, as sw_sweep runs them on a handle, with no handle and
 * no allocation.  Asynchronous on hip_stream (NULL: the null stream).
 *   params      dim, L, J, T, p_bond, seed as for sw_init; SW_PCC is refused,
 *               the other flags are ignored (the outputs below decide)
 *   dev_spins   device array of N int8 +1/-1, x fastest: the configuration
 *               before sweep sweep0 on entry, after sweep sweep0+n_sweeps-1
 *               on return (caller-owned, read and written in place,
 *               16-byte aligned)
 *   sweep0      index of the first sweep (keys the random stream)
 *   dev_series  NULL, or a device array of 2*n_sweeps int64: row k receives
 *               E_int and M after sweep sweep0+k (the call clears it first)
 *   dev_labels  NULL, or a device array of N int32: the canonical labels of
 *               the last sweep
 *   dev_err     NULL, or a device int32 the caller has zeroed: nonzero after
 *               the call completes if a device consistency check failed
 * Every other buffer comes from a static device array of 28 MiB per device
 * (held until the process ends), so lattices are limited to N <= 2^21 sites
 * (1448^2, 128^3): larger ones, and a null or misaligned spin array, give SW_EINVAL before
 * anything is enqueued.  All calls on one device share that array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  The results equal those of sw_init + sw_set_spins
 * (sweep0) + sw_sweep(n_sweeps) bit for bit.
 */
int sw_sweep_noalloc(const sw_params* params, int8_t* dev_spins, uint32_t sweep0, int32_t n_sweeps,
                     int64_t* dev_series, int32_t* dev_labels, int32_t* dev_err, void* hip_stream);

/* Release every resource the handle owns.  NULL is accepted. */
int sw_free(sw_lattice* h);

/* Thread-local description of the last failure (never NULL). */
const char* sw_last_error(void);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of simulation jobs                           */
/* ------------------------------------------------------------------------ */
typedef struct sw_server sw_server;

enum { SW_JOB_QUEUED = 0, SW_JOB_RUNNING = 1, SW_JOB_DONE = 2, SW_JOB_REJECTED = 3, SW_JOB_CANCELLED = 4 };

/*
 * Create a server that keeps at most max_slots lattices resident and whose
 * resident device footprint never exceeds hbm_budget_bytes (clamped to the
 * device memory free at creation).  A job whose allocation fails on
 * admission is rejected (SW_JOB_REJECTED); any other failure during admission
 * leaves it queued and is returned by sw_server_step.  Each tick
 * (sw_server_step) runs up to `sweeps_per_tick` sweeps of every resident job
 * in one batched launch, then retires finished jobs and admits queued ones.
 */
int sw_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t sweeps_per_tick,
                     int32_t device, void* hip_stream, sw_server** out);

/* Queue a job of n_sweeps sweeps.  Never blocks.  A job whose footprint alone
 * exceeds the budget is recorded as SW_JOB_REJECTED.  *job_id receives its id. */
int sw_server_submit(sw_server* s, const sw_params* p, int32_t n_sweeps, uint64_t* job_id);

/* Footprint in device bytes that a job with these parameters would hold. */
int sw_server_footprint(const sw_params* p, uint64_t* bytes);

/* State of a job (SW_JOB_*). */
int sw_server_poll(sw_server* s, uint64_t job_id, int32_t* state);

/* Result of a finished job: final (E_int, M), a 64-bit FNV-1a hash of its final
 * spins, and the submit / start / done times in seconds on the server clock. */
int sw_server_result(sw_server* s, uint64_t job_id, int64_t* e_int, int64_t* m, uint64_t* spin_hash,
                     double* t_submit, double* t_start, double* t_done);

/* Copy the final spins of a finished job (cap >= N). */
int sw_server_spins(sw_server* s, uint64_t job_id, int8_t* host_buf, int64_t cap);

/* Cancel a queued or running job; its slot and memory are released. */
int sw_server_cancel(sw_server* s, uint64_t job_id);

/* One tick: admit, sweep all resident jobs, retire.  *active receives the
 * number of jobs still queued or running afterwards (may be NULL). */
int sw_server_step(sw_server* s, int32_t* active);

/* Counters: jobs done, rejected, site-updates performed, device bytes in use. */
int sw_server_stats(sw_server* s, int64_t* done, int64_t* rejected, double* site_updates,
                    uint64_t* bytes_in_use);

/* Seconds on the server clock (monotonic, zero at creation). */
int sw_server_now(sw_server* s, double* t);

int sw_server_destroy(sw_server* s);

#ifdef __cplusplus
}
#endif

#if defined(SW_BUILD_LIBRARY) && defined(__GNUC__)
#pragma GCC visibility pop
#endif

#endif /* SW_API_H */
