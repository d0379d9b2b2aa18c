// sw_runtime.hpp -- host-side handle layout shared by the runtime, the
// autotuner and the job server (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sw_api.h"
#include "sw_device.hpp"
#include "sw_internal.hpp"

namespace sw {

struct ReplicaH {
    sw_params prm{};
    SwRep h{};               // host mirror of the device descriptor
    bool own_spins = true;
    bool labels_valid = false;
    bool dev_count_stale = false;   // plain sweeps advanced sweep / measured on the host only
};

struct TimedLaunch {
    int phase;
    hipEvent_t a, b;
};

// timed phases: 0 K1, 1 K2, 2 K3b, 3 PCC, 4 measurement, 5 batched sweeps, 6 K3a
constexpr int kPhases = 7;

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
uint64_t threshold_from_p(double p);
int validate_params(const sw_params* p);
uint64_t nsites_of(const sw_params* p);
int default_shape(int dim);
void fill_geometry(SwRep& h, int shape);
uint64_t footprint_bytes(const sw_params* p, int shape);
size_t spin_bytes(const SwRep& h);
int read_spins(const SwRep& m, int8_t* host_buf);
int replica_alloc(ReplicaH& r, const sw_params* p, int shape, hipStream_t stream);
void replica_free(ReplicaH& r);

}  // namespace sw

struct sw_lattice {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int mode = SW_MODE_PLAIN;
    int per_cu[3] = {8, 8, 8};          // plain-kernel workgroups per CU (K1, K2, K3)
    std::vector<sw::ReplicaH> reps;
    sw::SwRep* d_reps = nullptr;        // device descriptor array
    int32_t* err = nullptr;             // device consistency-check word shared by the replicas
    uint32_t* bar = nullptr;            // grid-barrier word of the persistent batched engine (same allocation)
    bool mirror_stale = false;          // device-side counters changed since the last read
    // timing
    bool timing = false;
    std::vector<sw::TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    double ms[sw::kPhases] = {};
    int64_t launches[sw::kPhases] = {};
    // batched execution (work list of all replicas' tiles, replayed graph)
    sw::EngineItem* items = nullptr;    // the work list, then the PCC candidate and slot lists
    size_t items_cap = 0;
    int nitems = 0;
    int ncand = 0;                       // PCC tiles on a hyperplane x_a = 0 (after the work list)
    int nperc = 0;                       // PCC slot chunks (after the candidate list)
    int nreplist = 0;                    // replicas of the groups (after the slot list)
    sw::BatchGroup groups[2] = {};       // the batch's groups (one dimension each)
    int ngroups = 0;
    hipStream_t side = nullptr;          // second stream of a batch of two groups
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    bool items_dirty = true;
    int batch_per_cu = 0;               // workgroups per CU of the batched phase launches (0: one per tile)
    int merge_width = 0;                // threads per tile of the border merge (0: the tile's default, 64, 256)
    int batch_engine = SW_ENGINE_GRAPH; // phase kernels replayed from a graph, or one persistent launch
    int persist_grid = 0;               // workgroups of the last persistent launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_n = -1;
    int graph_grid = -1;
    int graph_item_grid = -1;
    int graph_merge = -1;
    int graph_flags = -1;
    int graph_variant = -1;
};

namespace sw {
int handle_sync(sw_lattice* h);
int sync_mirror(sw_lattice* h);
int refresh_mirror(sw_lattice* h);
int push_desc(sw_lattice* h, int r);
int ensure_capacity(sw_lattice* h, int r, uint64_t need);
int plain_sweep(sw_lattice* h, int r, int32_t n);
int batched_sweep(sw_lattice* h, int32_t n);
int engine_variant(sw_lattice* h, int* variant);
int timing_collect(sw_lattice* h);
}  // namespace sw
