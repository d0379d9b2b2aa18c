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

struct EngineCtl {
    unsigned count;   // workgroups arrived at the current barrier
    unsigned gen;     // barrier generation
    int abort;        // set when a barrier wait timed out
    int nreps;        // replicas in the descriptor array
};

int device_cu_count();
uint64_t device_wallclock_hz();

int launch_k1(const SwRep& h, SwRep* d, uint32_t s, int64_t* em, hipStream_t stream, int per_cu);
int launch_k2(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream, int per_cu);
int launch_k3(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream, int per_cu);
int launch_cand(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream);
int launch_perc(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream);
int launch_measure(const SwRep& h, SwRep* d, int64_t* dst, hipStream_t stream);
int launch_init(const SwRep& h, SwRep* d, hipStream_t stream);
int launch_set_state(SwRep* d, uint32_t sweep, uint32_t measured, double p, uint64_t thr, int set_p,
                     hipStream_t stream);
int engine_grid_limit();
int launch_engine(SwRep* reps, const EngineItem* items, int nitems, EngineCtl* ctl, int n_sweeps, int any_pcc,
                  int any_series, int grid, uint64_t timeout_ticks, hipStream_t stream);

int shape_count(int dim);
int shape_extents(int dim, int id, int* tx, int* ty, int* tz);
int shape_xwords(int dim, int id);

}  // namespace sw
