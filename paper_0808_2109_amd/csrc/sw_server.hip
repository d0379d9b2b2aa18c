// sw_server.hip -- continuous-batching job server.
//
// Jobs (one lattice each, any dim / L / T / seed / sweep count) are queued on
// submit.  Each tick the server
//   1. admits queued jobs in arrival order while a slot is free and the
//      resident footprint stays within the memory budget,
//   2. runs up to `sweeps_per_tick` sweeps of every resident job as one
//      batched hipGraph launch (replayed while the resident set is
//      unchanged), each job stopping at its own sweep count,
//   3. retires finished jobs: records (E_int, M), the FNV-1a hash of the final
//      spins and the time stamps, and frees the slot.
// A job's random stream is keyed by its own seed and sweep index, never by
// its slot or by the other residents, so its result is bit-identical to the
// same job run alone.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "sw_runtime.hpp"

namespace sw {

struct Job {
    uint64_t id = 0;
    sw_params prm{};
    int32_t n_sweeps = 0;
    int32_t state = SW_JOB_QUEUED;
    int slot = -1;
    uint64_t bytes = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int64_t e_int = 0, m = 0;
    uint64_t hash = 0;
    std::vector<int8_t> spins;   // kept for jobs of up to kKeepSpins sites
};

constexpr uint64_t kKeepSpins = 1ull << 22;

static uint64_t fnv1a(const int8_t* p, size_t n)
{
    uint64_t h = 0xCBF29CE484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= (uint8_t)p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

}  // namespace sw

struct sw_server {
    std::mutex mu;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    int32_t max_slots = 0;
    int32_t tick = 1;
    sw_lattice* lat = nullptr;              // slot table: one replica per slot
    std::vector<uint64_t> slot_job;         // job id per slot (0 = free)
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, sw::Job> jobs;
    uint64_t next_id = 1;
    int64_t n_done = 0, n_rejected = 0;
    double site_updates = 0.0;
    std::chrono::steady_clock::time_point t0;
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

using namespace sw;

static int free_slot(sw_server* s, int slot)
{
    ReplicaH& r = s->lat->reps[slot];
    replica_free(r);
    std::memset(&r.h, 0, sizeof(r.h));
    r.h.active = 0;
    r.labels_valid = false;
    s->slot_job[slot] = 0;
    s->lat->items_dirty = true;
    return push_desc(s->lat, slot);
}

static int admit(sw_server* s)
{
    while (!s->queue.empty()) {
        Job& j = s->jobs[s->queue.front()];
        int slot = -1;
        for (int k = 0; k < s->max_slots; ++k)
            if (s->slot_job[k] == 0) {
                slot = k;
                break;
            }
        if (slot < 0 || s->in_use + j.bytes > s->budget) break;   // arrival order: no overtaking
        ReplicaH& r = s->lat->reps[slot];
        int rc = replica_alloc(r, &j.prm, default_shape(j.prm.dim), s->lat->stream);
        if (rc) {
            // the slot stays free (replica_alloc released what it took); the
            // device descriptor of the slot was never touched
            std::memset(&r.h, 0, sizeof(r.h));
            r.h.active = 0;
            if (rc != SW_ENOMEM) return rc;   // the job stays queued
            // the device could not hold the job even within the budget: it is
            // rejected rather than retried forever
            s->queue.pop_front();
            j.state = SW_JOB_REJECTED;
            j.t_done = s->now();
            s->n_rejected += 1;
            continue;
        }
        r.h.limit = (uint32_t)j.n_sweeps;
        r.h.active = 1;
        r.h.err = s->lat->err;
        r.labels_valid = false;
        rc = push_desc(s->lat, slot);
        if (!rc && launch_init(r.h, &s->lat->d_reps[slot], s->lat->stream)) rc = fail(SW_EHIP, "init launch failed");
        if (rc) {
            const int frc = free_slot(s, slot);   // the job stays queued
            return frc ? frc : rc;
        }
        s->queue.pop_front();
        s->slot_job[slot] = j.id;
        s->lat->items_dirty = true;
        s->in_use += j.bytes;
        j.slot = slot;
        j.state = SW_JOB_RUNNING;
        j.t_start = s->now();
    }
    return SW_OK;
}

static int retire(sw_server* s)
{
    int rc = sync_mirror(s->lat);
    if (rc) return rc;
    for (int k = 0; k < s->max_slots; ++k) {
        const uint64_t id = s->slot_job[k];
        if (!id) continue;
        ReplicaH& r = s->lat->reps[k];
        if (r.h.sweep < r.h.limit) continue;
        Job& j = s->jobs[id];
        rc = sw_measure(s->lat, k, &j.e_int, &j.m);
        if (rc) return rc;
        std::vector<int8_t> sp(r.h.N);
        rc = read_spins(r.h, sp.data());
        if (rc) return rc;
        j.hash = fnv1a(sp.data(), sp.size());
        if (r.h.N <= kKeepSpins) j.spins.swap(sp);
        j.state = SW_JOB_DONE;
        j.t_done = s->now();
        s->site_updates += (double)r.h.N * (double)j.n_sweeps;
        s->in_use -= j.bytes;
        s->n_done += 1;
        j.slot = -1;
        rc = free_slot(s, k);
        if (rc) return rc;
    }
    return SW_OK;
}

extern "C" {

int sw_server_footprint(const sw_params* p, uint64_t* bytes)
{
    int rc = validate_params(p);
    if (rc) return rc;
    if (!bytes) return fail(SW_EINVAL, "null output");
    sw_params q = *p;
    q.flags &= ~(uint32_t)SW_RECORD_SERIES;
    *bytes = footprint_bytes(&q, default_shape(q.dim));
    return SW_OK;
}

int sw_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t sweeps_per_tick, int32_t device,
                     void* hip_stream, sw_server** out)
{
    if (!out) return fail(SW_EINVAL, "null output");
    if (max_slots < 1 || max_slots > 65536) return fail(SW_EINVAL, "max_slots must be in [1, 65536]");
    if (sweeps_per_tick < 1) return fail(SW_EINVAL, "sweeps_per_tick must be >= 1");
    // the slot table is a lattice handle whose replicas start empty
    sw_params tiny;
    sw_params_default(&tiny);
    tiny.L = 3;
    std::vector<sw_params> ps((size_t)max_slots, tiny);
    sw_lattice* lat = nullptr;
    int rc = sw_init(ps.data(), max_slots, device, hip_stream, &lat);
    if (rc) return rc;
    sw_server* s = new (std::nothrow) sw_server();
    if (!s) {
        sw_free(lat);
        return fail(SW_ENOMEM, "host allocation failed");
    }
    s->lat = lat;
    s->lat->mode = SW_MODE_BATCHED;
    // the budget never exceeds the device memory free at creation
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (uint64_t)free_b < hbm_budget_bytes)
        hbm_budget_bytes = (uint64_t)free_b;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->tick = sweeps_per_tick;
    s->slot_job.assign((size_t)max_slots, 0);
    s->t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < max_slots && !rc; ++k) rc = free_slot(s, k);
    if (rc) {
        sw_server_destroy(s);
        return rc;
    }
    *out = s;
    return SW_OK;
}

int sw_server_submit(sw_server* s, const sw_params* p, int32_t n_sweeps, uint64_t* job_id)
{
    if (!s || !job_id) return fail(SW_EINVAL, "null argument");
    int rc = validate_params(p);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(SW_EINVAL, "negative sweep count");
    std::lock_guard<std::mutex> g(s->mu);
    Job j;
    j.id = s->next_id++;
    j.prm = *p;
    j.prm.flags &= ~(uint32_t)SW_RECORD_SERIES;
    j.n_sweeps = n_sweeps;
    j.bytes = footprint_bytes(&j.prm, default_shape(j.prm.dim));
    j.t_submit = s->now();
    if (j.bytes > s->budget) {
        j.state = SW_JOB_REJECTED;
        s->n_rejected += 1;
    } else {
        s->queue.push_back(j.id);
    }
    *job_id = j.id;
    s->jobs.emplace(j.id, std::move(j));
    return SW_OK;
}

int sw_server_poll(sw_server* s, uint64_t job_id, int32_t* state)
{
    if (!s || !state) return fail(SW_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SW_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    *state = it->second.state;
    return SW_OK;
}

int sw_server_result(sw_server* s, uint64_t job_id, int64_t* e_int, int64_t* m, uint64_t* spin_hash,
                     double* t_submit, double* t_start, double* t_done)
{
    if (!s) return fail(SW_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SW_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    const Job& j = it->second;
    if (j.state == SW_JOB_CANCELLED) return fail(SW_ECANCELLED, "job was cancelled");
    if (j.state != SW_JOB_DONE) return fail(SW_ESTATE, "job is not finished");
    if (e_int) *e_int = j.e_int;
    if (m) *m = j.m;
    if (spin_hash) *spin_hash = j.hash;
    if (t_submit) *t_submit = j.t_submit;
    if (t_start) *t_start = j.t_start;
    if (t_done) *t_done = j.t_done;
    return SW_OK;
}

int sw_server_spins(sw_server* s, uint64_t job_id, int8_t* host_buf, int64_t cap)
{
    if (!s || !host_buf) return fail(SW_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SW_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    const Job& j = it->second;
    if (j.state != SW_JOB_DONE) return fail(SW_ESTATE, "job is not finished");
    if (j.spins.empty()) return fail(SW_ESTATE, "spins are kept only for jobs of up to 2^22 sites");
    if (cap < (int64_t)j.spins.size()) return fail(SW_EINVAL, "buffer smaller than N");
    std::memcpy(host_buf, j.spins.data(), j.spins.size());
    return SW_OK;
}

int sw_server_cancel(sw_server* s, uint64_t job_id)
{
    if (!s) return fail(SW_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(SW_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    Job& j = it->second;
    if (j.state == SW_JOB_QUEUED) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == job_id) {
                s->queue.erase(q);
                break;
            }
    } else if (j.state == SW_JOB_RUNNING) {
        int rc = handle_sync(s->lat);
        if (rc) return rc;
        s->in_use -= j.bytes;
        rc = free_slot(s, j.slot);
        if (rc) return rc;
        j.slot = -1;
    } else {
        return fail(SW_ESTATE, "job already finished");
    }
    j.state = SW_JOB_CANCELLED;
    j.t_done = s->now();
    return SW_OK;
}

int sw_server_step(sw_server* s, int32_t* active)
{
    if (!s) return fail(SW_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    int rc = hipSetDevice(s->lat->device) == hipSuccess ? SW_OK : fail(SW_EHIP, "hipSetDevice");
    if (!rc) rc = admit(s);
    bool any = false;
    for (int k = 0; k < s->max_slots; ++k) any = any || s->slot_job[k] != 0;
    if (!rc && any) rc = batched_sweep(s->lat, s->tick);
    if (!rc) rc = retire(s);
    if (!rc) rc = admit(s);      // refill freed slots before the next tick
    if (rc) return rc;
    if (active) {
        int32_t n = (int32_t)s->queue.size();
        for (int k = 0; k < s->max_slots; ++k) n += s->slot_job[k] != 0;
        *active = n;
    }
    return SW_OK;
}

int sw_server_stats(sw_server* s, int64_t* done, int64_t* rejected, double* site_updates, uint64_t* bytes_in_use)
{
    if (!s) return fail(SW_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    if (done) *done = s->n_done;
    if (rejected) *rejected = s->n_rejected;
    if (site_updates) *site_updates = s->site_updates;
    if (bytes_in_use) *bytes_in_use = s->in_use;
    return SW_OK;
}

int sw_server_now(sw_server* s, double* t)
{
    if (!s || !t) return fail(SW_EINVAL, "null argument");
    *t = s->now();
    return SW_OK;
}

int sw_server_destroy(sw_server* s)
{
    if (!s) return SW_OK;
    if (s->lat) sw_free(s->lat);
    delete s;
    return SW_OK;
}

}  // extern "C"
