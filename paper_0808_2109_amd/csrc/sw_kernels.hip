// sw_kernels.hip -- the HIP kernels of the sweep and their host launchers.
//
// Plain path: one launch per phase and replica (K1, K2, [PCC candidates],
// K3a, K3b, [PCC coverage test and feedback]), each one workgroup per tile.  Batched path: each
// phase is one launch over the tiles of all replicas, and the launches of
// many sweeps are replayed from one hipGraph.
#include "sw_device.hpp"
#include "sw_internal.hpp"

namespace sw {

// tile shapes: (id, dim, TX, TY, TZ).  The batched kernels are compiled for
// the pairs (2D shape i, 3D shape i).
// Every shape has 64 rows (TY * TZ), one per lane of the K1 wave.
#define SW_SHAPES_2D(X) X(0, 2, 64, 64, 1) X(1, 2, 32, 64, 1)
#define SW_SHAPES_3D(X) X(0, 3, 32, 8, 8) X(1, 3, 64, 8, 8)
#define SW_SHAPES(X) SW_SHAPES_2D(X) SW_SHAPES_3D(X)
using Eng0_2D = TileCfg<2, 64, 64, 1>;
using Eng0_3D = TileCfg<3, 32, 8, 8>;
using Eng1_2D = TileCfg<2, 32, 64, 1>;
using Eng1_3D = TileCfg<3, 64, 8, 8>;
#define SW_ENGINE_PAIRS(X) X(0, Eng0_2D, Eng0_3D) X(1, Eng1_2D, Eng1_3D)

constexpr int kNumShapes = 2;

// XCD-aware chunking: workgroup b runs on XCD b % 8.  Giving XCD k the k-th
// eighth of the (replica, tile) work list keeps a band of neighbouring tiles
// (whose halos and labels are shared) inside one XCD's L2.
__device__ __forceinline__ void chunk_of(int nitems, int& i0, int& i1)
{
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int lam = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    i0 = (int)(((int64_t)lam * nitems) / G);
    i1 = (int)(((int64_t)(lam + 1) * nitems) / G);
}

__device__ __forceinline__ void block_sum2(int64_t& a, int64_t& b, int64_t* red)
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            a += red[2 * w];
            b += red[2 * w + 1];
        }
    }
}

// ---------------------------------------------------------------------------
// Plain kernels.
// ---------------------------------------------------------------------------
// sum of a and b over the wave, then one atomic add per wave
__device__ __forceinline__ void wave_flush_em(int64_t a, int64_t b, int64_t* dst)
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long*)&dst[0], (unsigned long long)a);
        atomicAdd((unsigned long long*)&dst[1], (unsigned long long)b);
    }
}

// K1: one workgroup of K1Cfg<C>::NT threads per tile, grid = ntiles; block b
// runs on XCD b % 8, which gets the b % 8-th eighth of the tiles
__device__ __forceinline__ int xcd_item(int nitems)
{
    int i0, i1;
    chunk_of(nitems, i0, i1);
    return i0;
}

// waves per SIMD asked of the compiler for K1: 64-wide tiles (four-wave
// workgroups) gain from an eighth wave even with scalar registers spilled to
// vector lanes; 32-wide tiles (two-wave workgroups) run better at fewer
template <class C>
constexpr int k1_waves() { return C::TX == 64 ? 8 : 6; }

template <class C, bool PCC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(k1_waves<C>()))) void k1_kernel(
    const SwRep* Rd, uint32_t s, int64_t* em)
{
    __shared__ K1Smem<C, PCC> sm;
    const SwRep R = *Rd;
    int64_t e = 0, m = 0;
    k1_tile<C, PCC>(R, xcd_item(R.ntiles), s, R.thr, sm, em != nullptr, e, m);
    if (em) wave_flush_em(e, m, em);
}

// K2: one workgroup per tile, grid = ntiles (XCD-aware order)
template <class C, int NT>
__global__ __launch_bounds__(NT) void k2_kernel(const SwRep* Rd)
{
    __shared__ K2Smem<C> sm;
    const SwRep R = *Rd;
    k2_tile<C, NT>(R, xcd_item(R.ntiles), sm);
}
// K3a: one wave per tile, grid = ntiles
template <class C>
__global__ __launch_bounds__(64) void k3a_kernel(const SwRep* Rd, uint32_t s)
{
    __shared__ K3aSmem<C> sm;
    const SwRep R = *Rd;
    CovArgs cov;
    k3a_tile<C>(R, xcd_item(R.ntiles), s, sm, cov);
    if (cov.nl >= 0) k3a_coverage(cov);
}

// K3b: one workgroup per tile, grid = ntiles (XCD-aware order)
template <class C>
__global__ __launch_bounds__(kK3Block) void k3_kernel(const SwRep* Rd, uint32_t s)
{
    __shared__ K3Smem<C> sm;
    const SwRep R = *Rd;
    k3_tile<C>(R, xcd_item(R.ntiles), s, sm);
}

template <class C>
__global__ __launch_bounds__(kBlock) void kcand_kernel(const SwRep* Rd, uint32_t s)
{
    const SwRep R = *Rd;
    int t0, t1;
    chunk_of(R.ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) k_cand_tile<C>(R, t, s);
}

// coverage test of the candidates' bitmaps (slots [c0, c1) of every axis);
// the bitmaps are cleared for the next sweep.  One wave per slot: its lanes
// read consecutive bitmap words, and a ballot tells whether every coordinate
// is covered (periodic box, extension rule) or, for an open box, whether the
// candidate (which touches coordinate 0) also touches coordinate L - 1.
__device__ void perc_chunk(const SwRep& R, uint32_t c0, uint32_t c1, int* local_flag)
{
    const uint32_t L = (uint32_t)R.L;
    const uint32_t bw = (L + 31u) / 32u;
    const uint32_t nslots = (R.dim == 3) ? L * L : L;
    const uint32_t tailbits = L & 31u;
    const uint32_t tailmask = tailbits ? ((1u << tailbits) - 1u) : 0xFFFFFFFFu;
    const bool open = (R.flags & FLAG_OPEN) != 0;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int a = 0; a < R.dim; ++a) {
        for (uint32_t c = c0 + wave; c < c1; c += nw) {   // wave-uniform
            uint32_t* bm = R.bmp + ((size_t)a * nslots + c) * bw;
            bool gap = false;                            // a coordinate of this lane's words is not covered
            for (uint32_t w = lane; w < bw; w += 64u) {
                const uint32_t v = bm[w];
                const uint32_t want = open ? ((w == bw - 1u) ? (1u << ((L - 1u) & 31u)) : 0u)
                                           : ((w == bw - 1u) ? tailmask : 0xFFFFFFFFu);
                gap = gap || (v & want) != want;
                if (v) bm[w] = 0;
            }
            if (!__ballot(gap) && lane == 0) *local_flag = 1;
        }
    }
}

// PCC feedback after sweep s: p -/+ dp, dp = dp0 * 2^-(s / halve_every),
// clamped to [0, 1]; the next sweep's threshold follows from p
__device__ void pcc_update(SwRep* Rd, uint32_t s)
{
    const int perc = __hip_atomic_exchange(Rd->pflag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double dp = ldexp(Rd->dp0, -(int)(s / Rd->halve_every));
    const double p = __longlong_as_double(
        (long long)__hip_atomic_load((unsigned long long*)&Rd->p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    double q = perc ? (p - dp) : (p + dp);
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    uint64_t thr;
    if (!(q > 0.0)) thr = 0;
    else if (q >= 1.0) thr = 4294967296ull;
    else thr = (uint64_t)floor(ldexp(q, 32));
    __hip_atomic_store((unsigned long long*)&Rd->p, (unsigned long long)__double_as_longlong(q), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store((unsigned long long*)&Rd->thr, (unsigned long long)thr, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if (s >= Rd->first && s - Rd->first < Rd->trace_cap) {
        Rd->perc_trace[s - Rd->first] = perc;
        Rd->p_trace[s - Rd->first] = q;
    }
}

__global__ __launch_bounds__(kBlock) void kperc_kernel(const SwRep* Rd)
{
    __shared__ int flag;
    const SwRep R = *Rd;
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    const uint32_t nslots = (R.dim == 3) ? (uint32_t)R.L * (uint32_t)R.L : (uint32_t)R.L;
    const uint32_t per = (nslots + gridDim.x - 1) / gridDim.x;
    const uint32_t c0 = min(nslots, blockIdx.x * per), c1 = min(nslots, c0 + per);
    perc_chunk(R, c0, c1, &flag);
    __syncthreads();
    if (threadIdx.x == 0 && flag) atomicOr(R.pflag, 1);
}

__global__ void kpcc_update_kernel(SwRep* Rd, uint32_t s)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) pcc_update(Rd, s);
}

// E_int and M of the current configuration, reading neighbours from memory
__device__ void measure_range(const SwRep& R, uint32_t i0, uint32_t i1, uint32_t stride, int64_t& e, int64_t& m)
{
    const uint32_t L = (uint32_t)R.L;
    const uint32_t LL = L * L;
    auto sp = [&](uint32_t j) { return 2 * (int)spin_up(R, j) - 1; };
    const bool open = (R.flags & FLAG_OPEN) != 0;     // no link wraps around the box
    for (uint32_t i = i0; i < i1; i += stride) {
        const int sv = sp(i);
        const uint32_t x = i % L;
        const uint32_t y = (i / L) % L;
        int nb = 0;
        if (!(open && x == L - 1)) nb += sp((x == L - 1) ? i - (L - 1) : i + 1);
        if (!(open && y == L - 1)) nb += sp((y == L - 1) ? i - (L - 1) * L : i + L);
        if (R.dim == 3) {
            const uint32_t z = i / LL;
            if (!(open && z == L - 1)) nb += sp((z == L - 1) ? i - (L - 1) * LL : i + LL);
        }
        m += sv;
        e += sv * nb;
    }
}

__global__ __launch_bounds__(kBlock) void kmeasure_kernel(const SwRep* Rd, int64_t* dst)
{
    __shared__ int64_t red[2 * kBlock / 64];
    const SwRep R = *Rd;
    int64_t e = 0, m = 0;
    measure_range(R, blockIdx.x * kBlock + threadIdx.x, R.N, gridDim.x * kBlock, e, m);
    block_sum2(e, m, red);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&dst[0], (unsigned long long)e);
        atomicAdd((unsigned long long*)&dst[1], (unsigned long long)m);
    }
}

// initial spins: site i is up when bit i%32 of word (i>>5)%4 of Philox(i>>7, 0, 0, INIT) is set.
// Bit-packed, word w of the lattice is word w%4 of block w>>2 (the bits past
// site N-1 cleared).
__global__ __launch_bounds__(kBlock) void kinit_kernel(const SwRep* Rd)
{
    const SwRep R = *Rd;
    if (R.flags & FLAG_BITPACK) {
        const uint32_t nw = (R.N + 31u) / 32u;
        uint32_t* words = reinterpret_cast<uint32_t*>(R.spins);
        for (uint32_t w = blockIdx.x * kBlock + threadIdx.x; w < nw; w += gridDim.x * kBlock) {
            const U4 r = philox10(w >> 2, 0u, 0u, kTagInit, (uint32_t)R.seed, (uint32_t)(R.seed >> 32));
            uint32_t v = pick(r, w & 3u);
            if (w == nw - 1u && (R.N & 31u)) v &= (1u << (R.N & 31u)) - 1u;
            words[w] = v;
        }
        return;
    }
    const uint32_t nblk = (R.N + 127u) / 128u;
    for (uint32_t b = blockIdx.x * kBlock + threadIdx.x; b < nblk; b += gridDim.x * kBlock) {
        const U4 r = philox10(b, 0u, 0u, kTagInit, (uint32_t)R.seed, (uint32_t)(R.seed >> 32));
        for (uint32_t k = 0; k < 128u; ++k) {
            const uint32_t i = b * 128u + k;
            if (i >= R.N) break;
            R.spins[i] = ((pick(r, k >> 5) >> (k & 31u)) & 1u) ? (int8_t)1 : (int8_t)-1;
        }
    }
}

__global__ void kset_state_kernel(SwRep* Rd, uint32_t sweep, uint32_t measured, uint32_t first, double p,
                                  uint64_t thr, int set_p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Rd->sweep = sweep;
        Rd->measured = measured;
        Rd->first = first;
        if (set_p) {
            Rd->p = p;
            Rd->thr = thr;
        }
    }
}

// ---------------------------------------------------------------------------
constexpr size_t cmax2(size_t a, size_t b) { return a > b ? a : b; }

// Batched execution: every phase of a sweep is one launch over the (replica,
// tile) work list of all replicas; a hipGraph holds the launches of n sweeps.
// Kernel boundaries order the phases, so no software grid barrier is needed.
// ---------------------------------------------------------------------------
// replica r runs sweep R.sweep + it in this graph when it is below its target
__device__ __forceinline__ bool rep_runs(const SwRep& R, int it, int n_sweeps, uint32_t& s)
{
    if (!R.active) return false;
    const uint64_t target = min((uint64_t)R.sweep + (uint64_t)n_sweeps, (uint64_t)R.limit);
    s = R.sweep + (uint32_t)it;
    return (uint64_t)s < target;
}

__device__ __forceinline__ void flush_em(int64_t e, int64_t m, int64_t* dst, int64_t* red)
{
    block_sum2(e, m, red);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&dst[0], (unsigned long long)e);
        atomicAdd((unsigned long long*)&dst[1], (unsigned long long)m);
    }
}

// K1 over the work list: one workgroup per item (grid = nitems, as many
// threads as the larger of the two tiles needs), with E, M of the incoming
// configuration added to the replica's series entry
// The per-item kernels below take either one workgroup per work item (grid =
// nitems, LOOP = false) or a smaller grid whose workgroups each run a
// contiguous, XCD-aware chunk of the list (LOOP = true); the results are the
// same for any grid.  The two are separate instantiations: with the item loop
// the compiler keeps far more registers live in the tile labelling.
template <bool LOOP>
__device__ __forceinline__ void item_range(int nitems, int& i0, int& i1)
{
    if (LOOP) {
        chunk_of(nitems, i0, i1);
    } else {
        i0 = xcd_item(nitems);
        i1 = i0 + 1;
    }
}

// One work item of each phase, shared by the phase kernels (one launch per
// phase) and the persistent kernel (all phases in one launch).
// (P2, P3: the PCC instantiation of the 2D / 3D tile labelling, chosen when
// a 2D / 3D PCC replica is active, so that the shared memory is sized for
// what the batch needs)
template <class C2, class C3, bool P2, bool P3>
__device__ __forceinline__ void k1_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps, char* smem)
{
    const SwRep R = reps[item.rep];   // a private copy: stores to the lattice's arrays cannot alias it
    uint32_t s;
    if (!rep_runs(R, it, n_sweeps, s)) return;
    int64_t* dst = nullptr;
    if ((R.flags & FLAG_SERIES) && s >= 1 && (it > 0 || R.measured < R.sweep))
        dst = R.series + 2 * (size_t)(s - 1 - R.first);
    int64_t e = 0, m = 0;
    if constexpr (std::is_same<C2, C3>::value && P2 == P3)   // a batch of one dimension: one copy of the tile code
        k1_tile<C2, P2>(R, item.tile, s, R.thr, *reinterpret_cast<K1Smem<C2, P2>*>(smem), dst != nullptr, e, m);
    else if (R.dim == 2)
        k1_tile<C2, P2>(R, item.tile, s, R.thr, *reinterpret_cast<K1Smem<C2, P2>*>(smem), dst != nullptr, e, m);
    else
        k1_tile<C3, P3>(R, item.tile, s, R.thr, *reinterpret_cast<K1Smem<C3, P3>*>(smem), dst != nullptr, e, m);
    if (dst) wave_flush_em(e, m, dst);
}

template <class C2, class C3, int NT>
__device__ __forceinline__ void k2_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps, char* smem)
{
    const SwRep R = reps[item.rep];   // a private copy: stores to the lattice's arrays cannot alias it
    uint32_t s;
    if (!rep_runs(R, it, n_sweeps, s)) return;
    if constexpr (std::is_same<C2, C3>::value) k2_tile<C2, NT>(R, item.tile, *reinterpret_cast<K2Smem<C2>*>(smem));
    else if (R.dim == 2) k2_tile<C2, NT>(R, item.tile, *reinterpret_cast<K2Smem<C2>*>(smem));
    else k2_tile<C3, NT>(R, item.tile, *reinterpret_cast<K2Smem<C3>*>(smem));
}

// PCC candidates of one tile of the candidate list
template <class C2, class C3>
__device__ __forceinline__ void kc_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps)
{
    const SwRep R = reps[item.rep];
    uint32_t s;
    if ((R.flags & (FLAG_PCC | FLAG_WIND)) != FLAG_PCC || !rep_runs(R, it, n_sweeps, s)) return;
    if constexpr (std::is_same<C2, C3>::value) k_cand_tile<C2>(R, item.tile, s);
    else if (R.dim == 2) k_cand_tile<C2>(R, item.tile, s);
    else k_cand_tile<C3>(R, item.tile, s);
}

// border-root resolution of one tile by one wave (smem: that wave's tables)
template <class C2, class C3>
__device__ __forceinline__ void k3a_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps, char* smem)
{
    const SwRep R = reps[item.rep];   // a private copy: stores to the lattice's arrays cannot alias it
    uint32_t s;
    if (!rep_runs(R, it, n_sweeps, s)) return;
    wave_lds_sync();   // the previous item's reads of the tables are done
    CovArgs cov;
    if constexpr (std::is_same<C2, C3>::value) k3a_tile<C2>(R, item.tile, s, *reinterpret_cast<K3aSmem<C2>*>(smem), cov);
    else if (R.dim == 2) k3a_tile<C2>(R, item.tile, s, *reinterpret_cast<K3aSmem<C2>*>(smem), cov);
    else k3a_tile<C3>(R, item.tile, s, *reinterpret_cast<K3aSmem<C3>*>(smem), cov);
    if (cov.nl >= 0) k3a_coverage(cov);
}

template <class C2, class C3>
__device__ __forceinline__ void k3_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps, char* smem)
{
    const SwRep R = reps[item.rep];   // a private copy: stores to the lattice's arrays cannot alias it
    uint32_t s;
    if (!rep_runs(R, it, n_sweeps, s)) return;
    if constexpr (std::is_same<C2, C3>::value) k3_tile<C2>(R, item.tile, s, *reinterpret_cast<K3Smem<C2>*>(smem));
    else if (R.dim == 2) k3_tile<C2>(R, item.tile, s, *reinterpret_cast<K3Smem<C2>*>(smem));
    else k3_tile<C3>(R, item.tile, s, *reinterpret_cast<K3Smem<C3>*>(smem));
}

// PCC coverage test of one item of the slot list: item (replica, k) stands
// for the candidate slots [k * kPercChunk, (k + 1) * kPercChunk) of every axis
// of that replica (the whole workgroup; pflag_local in shared memory)
__device__ __forceinline__ void perc_item(const SwRep* reps, const EngineItem& item, int it, int n_sweeps,
                                          int* pflag_local)
{
    const SwRep R = reps[item.rep];
    uint32_t s;
    if ((R.flags & (FLAG_PCC | FLAG_WIND)) != FLAG_PCC || !rep_runs(R, it, n_sweeps, s)) return;
    const uint32_t nslots = (R.dim == 3) ? (uint32_t)R.L * (uint32_t)R.L : (uint32_t)R.L;
    const uint32_t c0 = min(nslots, (uint32_t)item.tile * (uint32_t)kPercChunk);
    const uint32_t c1 = min(nslots, c0 + (uint32_t)kPercChunk);
    if (threadIdx.x == 0) *pflag_local = 0;
    __syncthreads();
    perc_chunk(R, c0, c1, pflag_local);
    __syncthreads();
    if (threadIdx.x == 0 && *pflag_local) atomicOr(R.pflag, 1);
}

// PCC feedback of replica r
__device__ __forceinline__ void update_rep(SwRep* reps, int r, int it, int n_sweeps)
{
    SwRep* Rp = &reps[r];
    uint32_t s;
    if (!(Rp->flags & FLAG_PCC) || !rep_runs(*Rp, it, n_sweeps, s)) return;
    pcc_update(Rp, s);
}

template <class C2, class C3, bool P2, bool P3, bool LOOP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(k1_waves<C2>()))) void kb1_kernel(
    SwRep* reps, const EngineItem* items, int nitems, int it, int n_sweeps)
{
    __shared__ __align__(16) char smem[cmax2(sizeof(K1Smem<C2, P2>), sizeof(K1Smem<C3, P3>))];
    int i0, i1;
    item_range<LOOP>(nitems, i0, i1);
    for (int i = i0; i < i1; ++i) k1_item<C2, C3, P2, P3>(reps, items[i], it, n_sweeps, smem);
}

// K2 over the work list
template <class C2, class C3, bool LOOP, int NT>
__global__ __launch_bounds__(NT) void kb2_kernel(SwRep* reps, const EngineItem* items, int nitems, int it,
                                                 int n_sweeps)
{
    __shared__ __align__(16) char smem[cmax2(sizeof(K2Smem<C2>), sizeof(K2Smem<C3>))];
    int i0, i1;
    item_range<LOOP>(nitems, i0, i1);
    for (int i = i0; i < i1; ++i) k2_item<C2, C3, NT>(reps, items[i], it, n_sweeps, smem);
}

// PCC candidates: one workgroup per item of the candidate list, which holds
// the tiles of PCC replicas that lie on a hyperplane x_a = 0
template <class C2, class C3>
__global__ __launch_bounds__(kBlock) void kbc_kernel(SwRep* reps, const EngineItem* items, int nitems, int it,
                                                     int n_sweeps)
{
    const int i = (int)blockIdx.x;
    if (i < nitems) kc_item<C2, C3>(reps, items[i], it, n_sweeps);
}

template <class C2, class C3, bool LOOP>
__global__ __launch_bounds__(64) void kb3a_kernel(SwRep* reps, const EngineItem* items, int nitems, int it,
                                                  int n_sweeps)
{
    __shared__ __align__(16) char smem[cmax2(sizeof(K3aSmem<C2>), sizeof(K3aSmem<C3>))];
    int i0, i1;
    item_range<LOOP>(nitems, i0, i1);
    for (int i = i0; i < i1; ++i) k3a_item<C2, C3>(reps, items[i], it, n_sweeps, smem);
}

template <class C2, class C3, bool LOOP>
__global__ __launch_bounds__(kK3Block) void kb3_kernel(SwRep* reps, const EngineItem* items, int nitems, int it,
                                                     int n_sweeps)
{
    __shared__ __align__(16) char smem[cmax2(sizeof(K3Smem<C2>), sizeof(K3Smem<C3>))];
    int i0, i1;
    item_range<LOOP>(nitems, i0, i1);
    for (int i = i0; i < i1; ++i) k3_item<C2, C3>(reps, items[i], it, n_sweeps, smem);
}

// PCC coverage test: one workgroup per item of the slot list
__global__ __launch_bounds__(kBlock) void kbp_kernel(SwRep* reps, const EngineItem* items, int nitems, int it,
                                                     int n_sweeps)
{
    __shared__ int pflag_local;
    const int i = (int)blockIdx.x;
    if (i < nitems) perc_item(reps, items[i], it, n_sweeps, &pflag_local);
}

// PCC feedback: one thread per replica
__global__ __launch_bounds__(kBlock) void kbu_kernel(SwRep* reps, int nreps, int it, int n_sweeps)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < nreps) update_rep(reps, r, it, n_sweeps);
}

// PCC feedback of the replicas of one group of a batch (their indices in list)
__global__ __launch_bounds__(kBlock) void kbu_list_kernel(SwRep* reps, const EngineItem* list, int n, int it,
                                                          int n_sweeps)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) update_rep(reps, list[i].rep, it, n_sweeps);
}

// E, M after the last sweep of every recording replica
__global__ __launch_bounds__(kBlock) void kbm_kernel(SwRep* reps, const EngineItem* items, int nitems, int n_sweeps)
{
    __shared__ int64_t red[2 * kBlock / 64];
    int i0, i1;
    chunk_of(nitems, i0, i1);
    int cur = -1;
    int64_t e = 0, m = 0;
    int64_t* dst = nullptr;
    for (int i = i0; i <= i1; ++i) {
        const int rep = (i < i1) ? items[i].rep : -2;
        if (rep != cur) {
            if (cur >= 0 && dst) flush_em(e, m, dst, red);
            e = m = 0;
            dst = nullptr;
            cur = rep;
            if (rep >= 0) {
                const SwRep& R = reps[rep];
                const uint64_t target = min((uint64_t)R.sweep + (uint64_t)n_sweeps, (uint64_t)R.limit);
                if (R.active && (R.flags & FLAG_SERIES) && target >= 1 && R.measured < target)
                    dst = R.series + 2 * (size_t)(target - 1 - R.first);
            }
        }
        if (i == i1) break;
        if (!dst) continue;
        const SwRep& R = reps[rep];
        // the tile's share of the site range
        const uint32_t a0 = (uint32_t)(((uint64_t)items[i].tile * R.N) / (uint32_t)R.ntiles);
        const uint32_t a1 = (uint32_t)(((uint64_t)(items[i].tile + 1) * R.N) / (uint32_t)R.ntiles);
        measure_range(R, a0 + threadIdx.x, a1, kBlock, e, m);
    }
}

// advance the sweep counters of the graph's n sweeps (last node)
__global__ __launch_bounds__(kBlock) void kbfin_kernel(SwRep* reps, int nreps, int n_sweeps)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nreps) return;
    SwRep* Rp = &reps[r];
    if (!Rp->active) return;
    const uint64_t target = min((uint64_t)Rp->sweep + (uint64_t)n_sweeps, (uint64_t)Rp->limit);
    if (Rp->flags & FLAG_SERIES) Rp->measured = (uint32_t)max((uint64_t)Rp->measured, target);
    Rp->sweep = (uint32_t)target;
}
// ---------------------------------------------------------------------------
// Persistent batched engine: one cooperative launch runs all n sweeps.  Every
// workgroup of the grid is resident at once; each walks its XCD-aware chunk
// of the work list phase by phase, and a software grid barrier stands where
// the phase kernels have a kernel boundary.  The barrier waits a bounded time:
// past it the workgroup sets ERR_BARRIER in the error word and every
// workgroup leaves at its next barrier, so the launch always ends.
// ---------------------------------------------------------------------------
struct PersistArgs {
    SwRep* reps;
    const EngineItem* items;
    const EngineItem* cand;
    const EngineItem* perc;
    uint32_t* bar;          // arrivals, zero at launch
    uint32_t* queue;        // one work counter per XCD, zero at launch
    int32_t* err;           // the handle's error word
    uint64_t limit;         // wall-clock ticks a workgroup waits at a barrier
    int nreps, nitems, ncand, nperc, n_sweeps, any_pcc;
};

// arrive, wait for the whole grid, then see every workgroup's writes; true
// when the launch is being abandoned
__device__ __forceinline__ bool grid_sync(const PersistArgs& A, uint32_t& target, int* abort_flag)
{
    __threadfence();   // this thread's writes are visible device-wide before it arrives
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(A.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        int ab = 0;
        while (__hip_atomic_load(A.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(A.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (1 << ERR_BARRIER)) {
                ab = 1;
                break;
            }
            if (wall_clock64() - t0 > A.limit) {
                atomicOr(A.err, 1 << ERR_BARRIER);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *abort_flag = ab;
    }
    __syncthreads();
    __threadfence();   // acquire: this workgroup's later loads see the others' writes
    return *abort_flag != 0;
}

// Dynamic work distribution: the work list is cut into one contiguous range
// per XCD (workgroup b runs on XCD b % 8, so neighbouring tiles stay in one
// L2), and the workgroups (or waves) of an XCD take the items of its range
// one at a time from a shared counter.  The counter only grows: every taker
// ends each phase with exactly one draw past the range, so after a phase the
// counter has grown by the range's length plus the number of takers, which
// every taker adds to its own copy of the base.
struct WorkQueue {
    uint32_t* ctr;
    uint32_t base;
    int lo, n;            // this XCD's range of the work list
    int block_takers;     // workgroups drawing from this counter
};

__device__ __forceinline__ WorkQueue make_queue(const PersistArgs& A)
{
    const int G = (int)gridDim.x;
    const int nq = (G % 8 == 0) ? 8 : 1;
    const int x = (int)blockIdx.x % nq;
    WorkQueue Q;
    Q.ctr = A.queue + x;
    Q.base = 0;
    Q.lo = (int)(((int64_t)x * A.nitems) / nq);
    Q.n = (int)(((int64_t)(x + 1) * A.nitems) / nq) - Q.lo;
    Q.block_takers = G / nq;
    return Q;
}

// next item for the whole workgroup, or -1 when the range is done
__device__ __forceinline__ int take_block(WorkQueue& Q, int* slot)
{
    __syncthreads();   // every thread has read the previous draw
    if (threadIdx.x == 0) *slot = (int)(atomicAdd(Q.ctr, 1u) - Q.base);
    __syncthreads();
    const int k = *slot;
    if (k >= Q.n) {
        Q.base += (uint32_t)(Q.n + Q.block_takers);
        return -1;
    }
    return Q.lo + k;
}

// next item for this wave alone, or -1 when the range is done
__device__ __forceinline__ int take_wave(WorkQueue& Q)
{
    uint32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(Q.ctr, 1u);
    const int k = (int)(__shfl(v, 0, 64) - Q.base);
    if (k >= Q.n) {
        Q.base += (uint32_t)(Q.n + Q.block_takers * (kBlock / 64));
        return -1;
    }
    return Q.lo + k;
}

template <class C2, class C3>
constexpr size_t k3a_slot() { return (cmax2(sizeof(K3aSmem<C2>), sizeof(K3aSmem<C3>)) + 15) & ~(size_t)15; }

template <class C2, class C3, bool P2, bool P3>
constexpr size_t persist_smem()
{
    return cmax2(cmax2(cmax2(sizeof(K1Smem<C2, P2>), sizeof(K1Smem<C3, P3>)),
                       cmax2(sizeof(K2Smem<C2>), sizeof(K2Smem<C3>))),
                 cmax2((kBlock / 64) * k3a_slot<C2, C3>(), cmax2(sizeof(K3Smem<C2>), sizeof(K3Smem<C3>))));
}

template <class C2, class C3, bool P2, bool P3>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void kpersist_kernel(PersistArgs A)
{
    static_assert(kK3Block == kBlock, "the flip phase runs on the persistent workgroup");
    __shared__ __align__(16) char smem[persist_smem<C2, C3, P2, P3>()];
    __shared__ int abort_flag, pflag_local, slot;
    uint32_t target = 0;
    WorkQueue Q = make_queue(A);
    const int wave = (int)threadIdx.x >> 6;
    for (int it = 0; it < A.n_sweeps; ++it) {
        for (int i; (i = take_block(Q, &slot)) >= 0;) k1_item<C2, C3, P2, P3>(A.reps, A.items[i], it, A.n_sweeps, smem);
        if (grid_sync(A, target, &abort_flag)) return;
        for (int i; (i = take_block(Q, &slot)) >= 0;) k2_item<C2, C3, kBlock>(A.reps, A.items[i], it, A.n_sweeps, smem);
        if (grid_sync(A, target, &abort_flag)) return;
        if (A.any_pcc && A.ncand > 0) {
            for (int i = (int)blockIdx.x; i < A.ncand; i += (int)gridDim.x)
                kc_item<C2, C3>(A.reps, A.cand[i], it, A.n_sweeps);
            if (grid_sync(A, target, &abort_flag)) return;
        }
        // one wave per tile, each wave with its own tables
        for (int i; (i = take_wave(Q)) >= 0;)
            k3a_item<C2, C3>(A.reps, A.items[i], it, A.n_sweeps, smem + wave * k3a_slot<C2, C3>());
        if (grid_sync(A, target, &abort_flag)) return;
        for (int i; (i = take_block(Q, &slot)) >= 0;) k3_item<C2, C3>(A.reps, A.items[i], it, A.n_sweeps, smem);
        if (grid_sync(A, target, &abort_flag)) return;
        if (A.any_pcc) {
            for (int i = (int)blockIdx.x; i < A.nperc; i += (int)gridDim.x)
                perc_item(A.reps, A.perc[i], it, A.n_sweeps, &pflag_local);
            if (grid_sync(A, target, &abort_flag)) return;
            for (int r = (int)(blockIdx.x * kBlock + threadIdx.x); r < A.nreps; r += (int)(gridDim.x * kBlock))
                update_rep(A.reps, r, it, A.n_sweeps);
            if (grid_sync(A, target, &abort_flag)) return;
        }
    }
}

// zero the barrier word and the per-XCD work counters
__global__ void kbar_reset_kernel(uint32_t* bar, uint32_t* queue)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *bar = 0u;
    if (blockIdx.x == 0 && threadIdx.x < 8) queue[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static int grid_for(int ntiles, int per_cu)
{
    const int cus = device_cu_count();
    int g = cus * per_cu;
    if (ntiles < g) g = ntiles;
    if (g >= 8) g -= g % 8;
    return g < 1 ? 1 : g;
}

#define SW_LAUNCH_CASE(id, D, X, Y, Z, KERNEL, ...)                                                    \
    case (D * 16 + id): {                                                                               \
        using C = TileCfg<D, X, Y, Z>;                                                                  \
        hipLaunchKernelGGL(KERNEL<C>, dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__);                \
        break;                                                                                          \
    }

int launch_k1(const SwRep& h, SwRep* d, uint32_t s, int64_t* em, hipStream_t stream, int per_cu)
{
    (void)per_cu;
    const int grid = h.ntiles;
    switch (h.dim * 16 + h.shape) {
#define L1(id, D, X, Y, Z)                                                                            \
    case (D * 16 + id): {                                                                            \
        using C = TileCfg<D, X, Y, Z>;                                                               \
        if (h.flags & FLAG_PCC)                                                                      \
            hipLaunchKernelGGL((k1_kernel<C, true>), dim3(grid), dim3(K1Cfg<C>::NT), 0, stream, d, s, em); \
        else                                                                                         \
            hipLaunchKernelGGL((k1_kernel<C, false>), dim3(grid), dim3(K1Cfg<C>::NT), 0, stream, d, s, em); \
        break;                                                                                       \
    }
        SW_SHAPES(L1)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// width: threads per tile of the border merge (64 or 256; 0: the tile's default)
int launch_k2(const SwRep& h, SwRep* d, hipStream_t stream, int width)
{
    const int grid = h.ntiles;
    switch (h.dim * 16 + h.shape) {
#define L2(id, D, X, Y, Z)                                                                   \
    case (D * 16 + id): {                                                                    \
        using C = TileCfg<D, X, Y, Z>;                                                       \
        const int w = width ? width : K2Cfg<C>::NT;                                          \
        if (w == 64) hipLaunchKernelGGL((k2_kernel<C, 64>), dim3(grid), dim3(64), 0, stream, d); \
        else hipLaunchKernelGGL((k2_kernel<C, kBlock>), dim3(grid), dim3(kBlock), 0, stream, d); \
        break;                                                                               \
    }
        SW_SHAPES(L2)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_k3a(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream)
{
    const int grid = h.ntiles;
    switch (h.dim * 16 + h.shape) {
#define L3A(id, D, X, Y, Z)                                                       \
    case (D * 16 + id): {                                                        \
        using C = TileCfg<D, X, Y, Z>;                                           \
        hipLaunchKernelGGL(k3a_kernel<C>, dim3(grid), dim3(64), 0, stream, d, s); \
        break;                                                                   \
    }
        SW_SHAPES(L3A)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_k3(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream, int per_cu)
{
    (void)per_cu;
    const int grid = h.ntiles;
    switch (h.dim * 16 + h.shape) {
#define L3(id, D, X, Y, Z)                                                               \
    case (D * 16 + id): {                                                               \
        using C = TileCfg<D, X, Y, Z>;                                                  \
        hipLaunchKernelGGL(k3_kernel<C>, dim3(grid), dim3(kK3Block), 0, stream, d, s);  \
        break;                                                                          \
    }
        SW_SHAPES(L3)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cand(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream)
{
    const int grid = h.ntiles;   // one tile per workgroup: only the tiles on x_a = 0 planes work
    switch (h.dim * 16 + h.shape) {
#define LC(id, D, X, Y, Z) SW_LAUNCH_CASE(id, D, X, Y, Z, kcand_kernel, d, s)
        SW_SHAPES(LC)
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// the percolation test (coverage bitmaps; the border merge itself flags a
// winding cluster) and the feedback step
int launch_perc(const SwRep& h, SwRep* d, uint32_t s, hipStream_t stream)
{
    if (h.flags & FLAG_WIND) {
        hipLaunchKernelGGL(kpcc_update_kernel, dim3(1), dim3(64), 0, stream, d, s);
        return hipGetLastError() == hipSuccess ? 0 : -3;
    }
    const uint32_t nslots = (h.dim == 3) ? (uint32_t)h.L * (uint32_t)h.L : (uint32_t)h.L;
    int grid = (int)((nslots + kBlock - 1) / kBlock);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(kperc_kernel, dim3(grid), dim3(kBlock), 0, stream, d);
    hipLaunchKernelGGL(kpcc_update_kernel, dim3(1), dim3(64), 0, stream, d, s);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_measure(const SwRep& h, SwRep* d, int64_t* dst, hipStream_t stream)
{
    int grid = (int)((h.N + kBlock - 1) / kBlock);
    const int cap = device_cu_count() * 8;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(kmeasure_kernel, dim3(grid), dim3(kBlock), 0, stream, d, dst);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_init(const SwRep& h, SwRep* d, hipStream_t stream)
{
    const uint32_t nblk = (h.N + 127u) / 128u;
    int grid = (int)((nblk + kBlock - 1) / kBlock);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(kinit_kernel, dim3(grid), dim3(kBlock), 0, stream, d);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_set_state(SwRep* d, uint32_t sweep, uint32_t measured, uint32_t first, double p, uint64_t thr, int set_p,
                     hipStream_t stream)
{
    hipLaunchKernelGGL(kset_state_kernel, dim3(1), dim3(64), 0, stream, d, sweep, measured, first, p, thr, set_p);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

struct BatchArgs {
    SwRep* reps;
    const EngineItem* items;
    const EngineItem* cand;
    const EngineItem* perc;
    int nreps, nitems, ncand, nperc, n_sweeps, any_pcc, ig, k2w;
    bool loop;
    hipStream_t stream;
};

// one sweep's phase launches over the work list for tile configurations CA and
// CB (2D and 3D); a batch whose replicas all have one dimension passes that
// dimension's configuration for both, so that the workgroups and the shared
// memory are sized for it alone
template <class CA, class CB, bool LP>
static void batch_phases(const BatchArgs& a, int it)
{
    const bool pcc2 = (a.any_pcc & 1) != 0, pcc3 = (a.any_pcc & 2) != 0;   // a 2D / 3D PCC replica is active
    const bool pa = (CA::D == 2) ? pcc2 : pcc3, pb = (CB::D == 2) ? pcc2 : pcc3;
    const dim3 g(a.ig), b1(max(K1Cfg<CA>::NT, K1Cfg<CB>::NT));
    if constexpr (std::is_same<CA, CB>::value) {
        if (pa) hipLaunchKernelGGL((kb1_kernel<CA, CB, true, true, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
        else hipLaunchKernelGGL((kb1_kernel<CA, CB, false, false, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
    } else {
        if (pa && pb)
            hipLaunchKernelGGL((kb1_kernel<CA, CB, true, true, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
        else if (pa)
            hipLaunchKernelGGL((kb1_kernel<CA, CB, true, false, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
        else if (pb)
            hipLaunchKernelGGL((kb1_kernel<CA, CB, false, true, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
        else
            hipLaunchKernelGGL((kb1_kernel<CA, CB, false, false, LP>), g, b1, 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
    }
    if (a.k2w == 64)
        hipLaunchKernelGGL((kb2_kernel<CA, CB, LP, 64>), g, dim3(64), 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
    else
        hipLaunchKernelGGL((kb2_kernel<CA, CB, LP, kBlock>), g, dim3(kBlock), 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
    if (a.any_pcc && a.ncand > 0)
        hipLaunchKernelGGL((kbc_kernel<CA, CB>), dim3(a.ncand), dim3(kBlock), 0, a.stream, a.reps, a.cand, a.ncand, it, a.n_sweeps);
    hipLaunchKernelGGL((kb3a_kernel<CA, CB, LP>), g, dim3(64), 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
    hipLaunchKernelGGL((kb3_kernel<CA, CB, LP>), g, dim3(kK3Block), 0, a.stream, a.reps, a.items, a.nitems, it, a.n_sweeps);
}

// the sweeps of one group of a batch (one dimension, tile C) on `stream`: each
// sweep's phases over the group's work list, then its PCC test and feedback
template <class C>
static void group_sweeps(BatchArgs a, const EngineItem* perc, int nperc, const EngineItem* reps_of, int nrep,
                         int merge_width, int item_grid)
{
    a.loop = item_grid < a.nitems;   // workgroups take chunks of the list
    a.ig = a.loop ? item_grid : a.nitems;
    a.k2w = merge_width ? merge_width : (C::D == 3 ? kBlock : K2Cfg<C>::NT);
    for (int it = 0; it < a.n_sweeps; ++it) {
        if (a.loop) batch_phases<C, C, true>(a, it);
        else batch_phases<C, C, false>(a, it);
        if (a.any_pcc) {
            if (nperc > 0)
                hipLaunchKernelGGL(kbp_kernel, dim3(nperc), dim3(kBlock), 0, a.stream, a.reps, perc, nperc, it, a.n_sweeps);
            hipLaunchKernelGGL(kbu_list_kernel, dim3((nrep + kBlock - 1) / kBlock), dim3(kBlock), 0, a.stream, a.reps,
                               reps_of, nrep, it, a.n_sweeps);
        }
    }
}

int launch_batch(int variant, SwRep* reps, int nreps, const EngineItem* items, int nitems, const EngineItem* cand_items,
                 const EngineItem* perc_items, const EngineItem* rep_list, const BatchGroup* groups, int ngroups,
                 int n_sweeps, int any_pcc, int any_series, int grid, int item_grid, int merge_width,
                 hipStream_t stream, hipStream_t side, hipEvent_t fork, hipEvent_t join)
{
    if (ngroups < 1 || ngroups > 2 || (ngroups == 2 && (!side || !fork || !join))) return -1;
    const int rgrid = (nreps + kBlock - 1) / kBlock;
    if (ngroups == 2) {   // the second group's stream starts after everything before the call
        if (hipEventRecord(fork, stream) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess) return -3;
    }
    for (int g = 0; g < ngroups; ++g) {
        const BatchGroup& G = groups[g];
        if (G.nitems <= 0) continue;
        BatchArgs a;
        a.reps = reps;
        a.items = items + G.item0;
        a.nitems = G.nitems;
        a.cand = cand_items + G.cand0;
        a.ncand = G.ncand;
        a.perc = perc_items + G.perc0;
        a.nperc = G.nperc;
        a.nreps = nreps;
        a.n_sweeps = n_sweeps;
        a.any_pcc = any_pcc;
        a.ig = 0;
        a.k2w = 0;
        a.loop = false;
        a.stream = (g == 0) ? stream : side;
        const EngineItem* perc = perc_items + G.perc0;
        const EngineItem* rl = rep_list + G.rep0;
        switch (variant) {
#define SW_GROUP(i, C2, C3)                                                                     \
    case i:                                                                                     \
        if (G.dim == 3) group_sweeps<C3>(a, perc, G.nperc, rl, G.nrep, merge_width, item_grid); \
        else group_sweeps<C2>(a, perc, G.nperc, rl, G.nrep, merge_width, item_grid);            \
        break;
            SW_ENGINE_PAIRS(SW_GROUP)
#undef SW_GROUP
            default: return -1;
        }
    }
    if (ngroups == 2) {   // and the first waits for the second
        if (hipEventRecord(join, side) != hipSuccess || hipStreamWaitEvent(stream, join, 0) != hipSuccess) return -3;
    }
    if (any_series) hipLaunchKernelGGL(kbm_kernel, dim3(grid), dim3(kBlock), 0, stream, reps, items, nitems, n_sweeps);
    hipLaunchKernelGGL(kbfin_kernel, dim3(rgrid), dim3(kBlock), 0, stream, reps, nreps, n_sweeps);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// the persistent kernel for the tile pair (C2, C3); a batch of one dimension
// passes that dimension's tile for both, so that the kernel carries one copy
// of the tile code and is sized for that tile alone
template <class C2, class C3>
static const void* persist_fn(bool pcc2, bool pcc3)
{
    if constexpr (std::is_same<C2, C3>::value) {
        const bool p = (C2::D == 2) ? pcc2 : pcc3;
        return p ? reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, true, true>)
                 : reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, false, false>);
    } else {
        if (pcc2 && pcc3) return reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, true, true>);
        if (pcc2) return reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, true, false>);
        if (pcc3) return reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, false, true>);
        return reinterpret_cast<const void*>(&kpersist_kernel<C2, C3, false, false>);
    }
}

// Sweeps per persistent launch: at most 4096, and few enough that the
// barrier's arrival count (at most 7 barriers a sweep, times the grid) and
// the work counters (4 phases a sweep, each the XCD's range plus one draw per
// taker) stay below 2^31.
static int persist_chunk(int nitems, int grid)
{
    const int64_t per_sweep = std::max<int64_t>(7ll * grid, 4ll * (nitems + 4ll * grid + 8));
    return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (int64_t(1) << 31) / per_sweep));
}

int launch_persistent(int variant, SwRep* reps, int nreps, const EngineItem* items, int nitems,
                      const EngineItem* cand_items, int ncand, const EngineItem* perc_items, int nperc, int n_sweeps,
                      int any_pcc, int any_series, int dims, int per_cu, uint32_t* bar, int32_t* err,
                      hipStream_t stream, int* grid_used)
{
    const bool pcc2 = (any_pcc & 1) != 0, pcc3 = (any_pcc & 2) != 0;
    const bool has2 = (dims & 1) != 0, has3 = (dims & 2) != 0;
    const void* fn = nullptr;
    switch (variant) {
#define SW_PERSIST(i, C2, C3)                                                                          \
    case i:                                                                                            \
        fn = (has2 && has3) ? persist_fn<C2, C3>(pcc2, pcc3)                                           \
                            : has3 ? persist_fn<C3, C3>(pcc2, pcc3) : persist_fn<C2, C2>(pcc2, pcc3); \
        break;
        SW_ENGINE_PAIRS(SW_PERSIST)
#undef SW_PERSIST
        default: return -1;
    }
    int dev = 0, resident = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, fn, kBlock, 0) != hipSuccess || resident < 1) return -3;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return -3;
    // every workgroup must be resident: at most `resident` per CU
    const int cus = device_cu_count();
    int grid = cus * ((per_cu > 0 && per_cu < resident) ? per_cu : resident);
    if (grid > nitems) grid = nitems;
    if (grid >= 8) grid -= grid % 8;
    if (grid < 1) grid = 1;
    PersistArgs a;
    a.reps = reps;
    a.items = items;
    a.cand = cand_items;
    a.perc = perc_items;
    a.bar = bar;
    a.queue = bar + 16;
    a.err = err;
    a.limit = (uint64_t)khz * 1000ull * 10ull;   // 10 s at a barrier
    a.nreps = nreps;
    a.nitems = nitems;
    a.ncand = ncand;
    a.nperc = nperc;
    a.any_pcc = any_pcc;
    const int rgrid = (nreps + kBlock - 1) / kBlock;
    const int chunk = persist_chunk(nitems, grid);
    for (int done = 0; done < n_sweeps;) {
        const int n = min(chunk, n_sweeps - done);
        a.n_sweeps = n;
        hipLaunchKernelGGL(kbar_reset_kernel, dim3(1), dim3(64), 0, stream, bar, a.queue);
        void* args[] = {&a};
        if (hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, stream) != hipSuccess) return -3;
        if (any_series) hipLaunchKernelGGL(kbm_kernel, dim3(grid), dim3(kBlock), 0, stream, reps, items, nitems, n);
        hipLaunchKernelGGL(kbfin_kernel, dim3(rgrid), dim3(kBlock), 0, stream, reps, nreps, n);
        done += n;
    }
    if (grid_used) *grid_used = grid;
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int shape_count(int dim)
{
    (void)dim;
    return kNumShapes;
}

int shape_extents(int dim, int id, int* tx, int* ty, int* tz)
{
#define SW_EXT(i, D, X, Y, Z)          \
    if (dim == D && id == i) {         \
        *tx = X;                       \
        *ty = Y;                       \
        *tz = Z;                       \
        return 0;                      \
    }
    SW_SHAPES(SW_EXT)
    return -1;
}

int shape_xwords(int dim, int id)
{
#define SW_XW(i, D, X, Y, Z) \
    if (dim == D && id == i) return TileCfg<D, X, Y, Z>::XW;
    SW_SHAPES(SW_XW)
    return -1;
}

int shape_fbw(int dim, int id)
{
#define SW_FBW(i, D, X, Y, Z) \
    if (dim == D && id == i) return TileCfg<D, X, Y, Z>::FBW;
    SW_SHAPES(SW_FBW)
    return -1;
}

int shape_ft(int dim, int id)
{
#define SW_FT(i, D, X, Y, Z) \
    if (dim == D && id == i) return TileCfg<D, X, Y, Z>::FT;
    SW_SHAPES(SW_FT)
    return -1;
}

}  // namespace sw
