// sw_internal.hpp -- declarations shared by the kernel launchers and the host
// runtime of libswgpu.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

struct SwRep;

struct EngineItem {
    int32_t rep;
    int32_t tile;
};

constexpr int kPercChunk = 64;   // candidate slots per workgroup of the batched coverage test

int device_cu_count();
uint64_t device_wallclock_hz();

int launch_k1(const SwRep& h, SwRep* d, uint32_t s, int64_t* em, hipStream_t stream, int per_cu);
int launch_k2(const SwRep& h, SwRep* d, hipStream_t stream, int width);
int launch_k3a(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream);
int launch_k3(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream, int per_cu);
int launch_cand(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream);
int launch_perc(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream);
int launch_measure(const SwRep& h, SwRep* d, int64_t* dst, hipStream_t stream);
int launch_init(const SwRep& h, SwRep* d, hipStream_t stream);
int launch_set_state(SwRep* d, uint32_t sweep, uint32_t measured, uint32_t first, double p, uint64_t thr, int set_p,
                     hipStream_t stream);
// enqueue n sweeps of every active replica as batched phase launches (used
// under stream capture to build the batch graph)
// (any_pcc: bit 0 a 2D PCC replica is active, bit 1 a 3D one; grid:
// workgroups of the list-chunking kernels; item_grid: workgroups of the
// per-tile phase kernels, nitems for one workgroup per work item)
// cand_items: the tiles of PCC replicas on a hyperplane x_a = 0; perc_items:
// (replica, k) for the candidate slots [k * kPercChunk, (k + 1) * kPercChunk)
// A batch runs as one or two groups of replicas, each of one dimension; each
// group's work items, candidate tiles, slot chunks and replicas are a
// contiguous range of its list.  Two groups run on two streams (forked from
// and joined back to the first), so that their phases may overlap.
struct BatchGroup {
    int item0, nitems;     // work list
    int cand0, ncand;      // PCC candidate list
    int perc0, nperc;      // PCC slot list
    int rep0, nrep;        // replica list
    int dim;
};
int launch_batch(int variant, SwRep* reps, int nreps, const EngineItem* items, int nitems, const EngineItem* cand_items,
                 const EngineItem* perc_items, const EngineItem* rep_list, const BatchGroup* groups, int ngroups,
                 int n_sweeps, int any_pcc, int any_series, int grid, int item_grid, int merge_width,
                 hipStream_t stream, hipStream_t side, hipEvent_t fork, hipEvent_t join);
// all n sweeps of a batch in persistent launches (one per 4096 sweeps) of
// co-resident workgroups, per_cu of them per CU (0: as many as fit); bar: a
// device word the launches use as their barrier; grid_used: the grid
int launch_persistent(int variant, SwRep* reps, int nreps, const EngineItem* items, int nitems,
                      const EngineItem* cand_items, int ncand, const EngineItem* perc_items, int nperc, int n_sweeps,
                      int any_pcc, int any_series, int dims, int per_cu, uint32_t* bar, int32_t* err,
                      hipStream_t stream, int* grid_used);

int shape_count(int dim);
int shape_extents(int dim, int id, int* tx, int* ty, int* tz);
int shape_xwords(int dim, int id);
int shape_fbw(int dim, int id);
int shape_ft(int dim, int id);

}  // namespace sw
