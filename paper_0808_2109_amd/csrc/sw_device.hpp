// sw_device.hpp -- device-side data layout and the per-tile phases of one
// Swendsen-Wang sweep (Lin & Zheng, Sec. I steps 1-3) on gfx950.
//
// A replica's lattice is cut into tiles of TX x TY (x TZ) sites, TX = 32 or
// 64, so that every wave64 covers whole tile rows.  One sweep is
//   K1  per tile: load the spins (+ the far halo) as one bit mask per row,
//       draw the bonds of the tile's own links from Philox as bit masks, label
//       the tile's clusters in LDS (runs along x from the bond masks, a
//       union-find over the remaining links), write a 16-bit tile-local label
//       per site and the bits of the tile's open links that leave it.  The
//       tile plays the part of a domain of Sec. II.
//   K2  per tile: join, in a global union-find over tile-local roots, the two
//       ends of every open link that leaves the tile (the border
//       reconciliation of Sec. II, in one pass instead of the master's second
//       labelling or the iterated neighbour exchange), and write this sweep's
//       flip-bit table.
//   K3  per tile: resolve every tile-local root once to its cluster root (the
//       smallest site index of the cluster: the label identity that the
//       min-label rule of Sec. II.B converges to) and give every site its
//       cluster's new spin (Sec. I step 3).
// plus the extension-rule percolation test and p feedback of Sec. III.
//
// Every union hooks the larger root under the smaller one, so the final roots
// do not depend on the order of unions, the tile shape or the schedule: the
// result is bit-identical to a sequential labelling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr uint32_t kTagInit = 0, kTagBond = 1, kTagRefine = 2, kTagFlip = 3;
constexpr uint32_t kBorderFlag = 0x8000u;

enum : uint32_t { FLAG_SERIES = 1u, FLAG_KEEP = 2u, FLAG_PCC = 4u };

// --------------------------------------------------------------------------
// Replica descriptor (device resident; the host keeps a mirror).
// --------------------------------------------------------------------------
struct SwRep {
    int32_t dim, L;
    uint32_t N;                 // L^dim < 2^31
    int32_t shape;              // tile shape id (per dim)
    int32_t tx, ty, tz;         // tile extents
    int32_t ntx, nty, ntz, ntiles;
    int32_t xwords;             // crossing-bit words per tile
    uint32_t flags;
    uint64_t seed;
    uint64_t thr;               // threshold of the next sweep (<= 2^32)
    double p;                   // bond probability of the next sweep
    double dp0;                 // PCC step at sweep 0
    uint32_t halve_every;       // PCC: dp halves every this many sweeps
    uint32_t sweep;             // sweeps done
    uint32_t limit;             // batched mode: never run past this sweep
    uint32_t measured;          // series entries complete (E,M after sweep k, k < measured)
    uint32_t series_cap;        // entries the series buffer holds
    uint32_t trace_cap;         // entries the PCC trace buffers hold
    int32_t active;             // batched mode: replica takes part
    int32_t pad0;
    int8_t* spins;              // N
    uint16_t* lab16;            // N tile-local labels | border flag
    int32_t* par;               // N global union-find parents (border roots only)
    int32_t* lab32;             // N final labels (FLAG_KEEP or FLAG_PCC), else null
    uint32_t* xbits;            // ntiles * xwords crossing-link bits
    uint32_t* fliptab;          // 4 * ceil(N/128) words: this sweep's flip bits
    int64_t* series;            // 2 * series_cap
    int64_t* acc;               // 2 scratch accumulators (measure)
    uint64_t* cand;             // PCC: dim * N candidate marks (tag << 32 | ~slot)
    uint32_t* bmp;              // PCC: dim * L^(dim-1) * ceil(L/32) coverage bitmaps
    int32_t* pflag;             // PCC: percolation flag of the current sweep
    int32_t* perc_trace;        // PCC: trace_cap flags
    double* p_trace;            // PCC: trace_cap values of p after each update
    int32_t* err;               // consistency-check bits (shared by a handle's replicas)
};

// consistency checks on data-dependent indices: a violation sets a bit that
// the host turns into an error instead of letting the access go out of range
enum : int { ERR_TILE_LABEL = 1, ERR_PARENT = 2, ERR_SLOT = 3 };

__device__ __forceinline__ void flag_error(const SwRep& R, int code)
{
    if (R.err) atomicOr(R.err, 1 << code);
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): the counter-based generator all draws
// of the method come from.  Ten rounds of the two-multiplier S-box; the key
// advances by the two Weyl constants between rounds.
// --------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = c0 * 0xD2511F53u;
        const uint32_t hi0 = __umulhi(c0, 0xD2511F53u);
        const uint32_t lo1 = c2 * 0xCD9E8D57u;
        const uint32_t hi1 = __umulhi(c2, 0xCD9E8D57u);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const U4& r, uint32_t w)
{
    return w == 0 ? r.x : w == 1 ? r.y : w == 2 ? r.z : r.w;
}

// --------------------------------------------------------------------------
// Tile shapes.
// --------------------------------------------------------------------------
template <int D_, int TX_, int TY_, int TZ_>
struct TileCfg {
    static constexpr int D = D_, TX = TX_, TY = TY_, TZ = TZ_;
    static constexpr int TS = TX * TY * TZ;
    static constexpr int NR = TY * TZ;                                // tile rows
    static constexpr int NRH = (D == 3) ? (TY + 1) * (TZ + 1) : TY + 1;  // rows incl. the +y / +z halo
    static constexpr int RPW = 64 / TX;                               // rows per wave64
    static constexpr int LOADIT = (NRH + 4 * RPW - 1) / (4 * RPW);    // row loads per lane
    static constexpr int SITEIT = TS / kBlock;                        // sites per thread
    static constexpr int F0 = TY * TZ, F1 = TX * TZ, F2 = (D == 3) ? TX * TY : 0;
    static constexpr int W0 = (F0 + 31) / 32, W1 = (F1 + 31) / 32, W2 = (F2 + 31) / 32;
    static constexpr int XW = W0 + W1 + W2;
    static constexpr int NB = TX / 16;        // Philox bond blocks per aligned row
    static_assert(TX == 32 || TX == 64, "a wave64 covers whole tile rows");
    static_assert(TS % kBlock == 0, "whole sites per thread");
    static_assert(NR <= kBlock, "one thread per row for the halo column");
    static_assert(TS <= 32768, "tile-local labels are 15-bit");
};

struct TileGeo {
    int x0, y0, z0, wx, wy, wz;
};

template <class C>
__device__ __forceinline__ TileGeo tile_geo(const SwRep& R, int t)
{
    TileGeo g;
    const int ix = t % R.ntx;
    const int iy = (t / R.ntx) % R.nty;
    const int iz = t / (R.ntx * R.nty);
    g.x0 = ix * C::TX;
    g.y0 = iy * C::TY;
    g.z0 = (C::D == 3) ? iz * C::TZ : 0;
    g.wx = min(C::TX, R.L - g.x0);
    g.wy = min(C::TY, R.L - g.y0);
    g.wz = (C::D == 3) ? min(C::TZ, R.L - g.z0) : 1;
    return g;
}

// global index of the tile-local site lr of the tile with origin (x0,y0,z0)
template <class C>
__device__ __forceinline__ uint32_t local_to_global(uint32_t lr, int x0, int y0, int z0, int L)
{
    const uint32_t lx = lr % C::TX;
    const uint32_t ly = (lr / C::TX) % C::TY;
    const uint32_t lz = lr / (C::TX * C::TY);
    return (uint32_t)(x0 + lx) + (uint32_t)L * ((uint32_t)(y0 + ly) + (uint32_t)L * (uint32_t)(z0 + lz));
}

// global root of the tile-local label stored for site gi
template <class C>
__device__ __forceinline__ uint32_t tile_root_of(const SwRep& R, uint32_t gi, uint32_t v)
{
    const uint32_t L = (uint32_t)R.L;
    const uint32_t x = gi % L;
    const uint32_t y = (gi / L) % L;
    const uint32_t z = (C::D == 3) ? gi / (L * L) : 0;
    const int x0 = (int)(x / C::TX) * C::TX;
    const int y0 = (int)(y / C::TY) * C::TY;
    const int z0 = (C::D == 3) ? (int)(z / C::TZ) * C::TZ : 0;
    const uint32_t lr = v & 0x7FFFu;
    const uint32_t r = (lr < (uint32_t)C::TS) ? local_to_global<C>(lr, x0, y0, z0, (int)L) : 0xFFFFFFFFu;
    if (r > gi) {            // a tile root precedes every site of its cluster
        flag_error(R, ERR_TILE_LABEL);
        return 0xFFFFFFFFu;
    }
    return r;
}

__device__ __forceinline__ uint64_t low_bits(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// --------------------------------------------------------------------------
// Union-find primitives.  Parents only ever point to smaller indices of the
// same cluster, so the root of a cluster is its smallest member.  A find may
// shorten paths with plain stores (every store writes an ancestor); a union
// hooks with an atomic min and retries from the value it displaced.
// --------------------------------------------------------------------------
__device__ __forceinline__ int lds_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(int* par, int x)
{
    while (true) {
        const int p = lds_load(&par[x]);
        if (p == x) return x;
        const int gp = lds_load(&par[p]);
        if (gp == p) return p;
        lds_store(&par[x], gp);
        x = gp;
    }
}

// root of x without writing: safe while other threads replace parents by
// roots (every value it can read is an ancestor of x)
__device__ __forceinline__ int lds_root(const int* par, int x)
{
    int p = lds_load(&par[x]);
    while (p != x) {
        x = p;
        p = lds_load(&par[x]);
    }
    return x;
}

__device__ __forceinline__ void lds_unite(int* par, int a, int b)
{
    while (true) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&par[b], a);
        if (old == b) return;
        b = old;
    }
}

__device__ __forceinline__ int g_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void g_store(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// parents are checked against [0, x]: a value outside it can only come from a
// broken invariant; it is reported and the chase stops (returns -1)
__device__ __forceinline__ int g_find(const SwRep& R, int* par, int x)
{
    while (true) {
        const int p = g_load(&par[x]);
        if (p == x) return x;
        if (p < 0 || p > x) {
            flag_error(R, ERR_PARENT);
            return -1;
        }
        const int gp = g_load(&par[p]);
        if (gp == p) return p;
        if (gp < 0 || gp > p) {
            flag_error(R, ERR_PARENT);
            return -1;
        }
        g_store(&par[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void g_unite(const SwRep& R, int* par, int a, int b)
{
    while (true) {
        a = g_find(R, par, a);
        b = g_find(R, par, b);
        if (a < 0 || b < 0) return;
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = __hip_atomic_fetch_min(&par[b], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == b) return;
        b = old;
    }
}

// read-only find, for phases that run after all unions are complete
__device__ __forceinline__ uint32_t ro_find(const SwRep& R, uint32_t x)
{
    int p = R.par[x];
    while ((uint32_t)p != x) {
        if (p < 0 || (uint32_t)p > x) {
            flag_error(R, ERR_PARENT);
            return x;
        }
        x = (uint32_t)p;
        p = R.par[x];
    }
    return x;
}

// --------------------------------------------------------------------------
// K1: bonds + tile labelling.
// --------------------------------------------------------------------------
template <class C>
struct K1Smem {
    int32_t par[C::TS];
    uint64_t S[C::NRH];        // spin-up bit masks of the rows (bit x), incl. the +y / +z halo rows
    uint64_t OPN[C::D][C::NR]; // open-bond masks of the tile's own links, per direction and row
    uint64_t RR[C::NR];        // x-runs: open x-bonds that stay inside the tile
    uint8_t HB[C::NRH];        // spin-up bit of the +x halo site of each row
    uint8_t flag[C::TS];
};

// equal-spin masks of a row's own links in direction d (bit x: link (x, d))
template <class C>
__device__ __forceinline__ uint64_t eq_mask(const K1Smem<C>& sm, int ly, int lz, int d, int wx)
{
    const int hr = ly + (C::TY + 1) * lz;
    const uint64_t s = sm.S[hr];
    uint64_t nb;
    if (d == 0) nb = (s >> 1) | ((uint64_t)sm.HB[hr] << (wx - 1));
    else if (d == 1) nb = sm.S[hr + 1];
    else nb = sm.S[hr + C::TY + 1];
    return ~(s ^ nb) & low_bits(wx);
}

template <class C>
__device__ void k1_tile(const SwRep& R, int t, uint32_t s, uint64_t thr, K1Smem<C>& sm, bool measure,
                        int64_t& e_acc, int64_t& m_acc)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const TileGeo g = tile_geo<C>(R, t);
    const int L = R.L;
    const uint32_t N = R.N;
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);

    // 1) spins as bit masks: rows of the tile, the +y halo row(s), the +z halo
    //    plane, and the +x halo site of every row
    {
        int8_t v[C::LOADIT];
        const int x = lane % C::TX;
        int hb = 0;
        if (tid < C::NR) {
            const int ly = tid % C::TY, lz = tid / C::TY;
            if (ly < g.wy && lz < g.wz) {
                const int gx = (g.x0 + g.wx == L) ? 0 : g.x0 + g.wx;
                hb = R.spins[(uint32_t)gx + (uint32_t)L * ((uint32_t)(g.y0 + ly) + (uint32_t)L * (uint32_t)(g.z0 + lz))] > 0;
            }
        }
#pragma unroll
        for (int i = 0; i < C::LOADIT; ++i) {
            const int hr = (wave + 4 * i) * C::RPW + lane / C::TX;
            const int hy = hr % (C::TY + 1), hz = hr / (C::TY + 1);
            bool need = hr < C::NRH && x < g.wx && hy <= g.wy;
            if (C::D == 3) need = need && hz <= g.wz && !(hy == g.wy && hz == g.wz);
            v[i] = 0;
            if (need) {
                int gy = g.y0 + hy, gz = g.z0 + hz;
                if (gy == L) gy = 0;
                if (C::D == 3 && gz == L) gz = 0;
                v[i] = R.spins[(uint32_t)(g.x0 + x) + (uint32_t)L * ((uint32_t)gy + (uint32_t)L * (uint32_t)gz)];
            }
        }
#pragma unroll
        for (int i = 0; i < C::LOADIT; ++i) {
            const int hr = (wave + 4 * i) * C::RPW + lane / C::TX;
            const uint64_t b = __ballot(v[i] > 0);
            if (x == 0 && hr < C::NRH) sm.S[hr] = (b >> (lane - x)) & low_bits(C::TX);
        }
        if (tid < C::NR) {
            const int ly = tid % C::TY, lz = tid / C::TY;
            sm.HB[ly + (C::TY + 1) * lz] = (uint8_t)hb;
#pragma unroll
            for (int d = 0; d < C::D; ++d) sm.OPN[d][tid] = 0;
        }
        for (int k = tid; k < C::TS; k += kBlock) sm.flag[k] = 0;
    }
    __syncthreads();

    // 2) bonds of the tile's own links (i, d), d < D: Philox blocks of 16 links
    //    give the high byte a of u; ties with thr>>24 draw the low 24 bits
    {
        const uint32_t t_hi = (uint32_t)(thr >> 24);
        const uint32_t t_lo = (uint32_t)(thr & 0xFFFFFFu);
        const int nslot = (L % 16 == 0) ? C::NB : C::NB + 1;
        const int nitems = C::D * C::NR * nslot;
        for (int it = tid; it < nitems; it += kBlock) {
            const int j = it % nslot;
            const int r = (it / nslot) % C::NR;
            const int d = it / (nslot * C::NR);
            const int ly = r % C::TY, lz = r / C::TY;
            if (ly >= g.wy || lz >= g.wz) continue;
            const uint32_t rowbase = (uint32_t)d * N + (uint32_t)g.x0 +
                                     (uint32_t)L * ((uint32_t)(g.y0 + ly) + (uint32_t)L * (uint32_t)(g.z0 + lz));
            const uint32_t blk = (rowbase >> 4) + (uint32_t)j;
            if (blk * 16u >= rowbase + (uint32_t)g.wx) continue;
            const uint64_t eq = eq_mask<C>(sm, ly, lz, d, g.wx);
            const U4 q = philox10(blk, 0u, s, kTagBond, k0, k1);
            uint64_t op = 0;
            uint32_t ties = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int x = (int)(blk * 16u + (uint32_t)k - rowbase);
                if (x < 0 || x >= g.wx) continue;
                if (!((eq >> x) & 1ull)) continue;
                const uint32_t word = (k < 4) ? q.x : (k < 8) ? q.y : (k < 12) ? q.z : q.w;
                const uint32_t a = (word >> (8 * (k & 3))) & 0xFFu;
                if (a < t_hi) op |= 1ull << x;
                if (a == t_hi) ties |= 1u << k;
            }
            while (ties) {
                const int k = __ffs(ties) - 1;
                ties &= ties - 1u;
                const uint32_t l = blk * 16u + (uint32_t)k;
                const U4 q2 = philox10(l >> 2, 0u, s, kTagRefine, k0, k1);
                if ((pick(q2, l & 3u) & 0xFFFFFFu) < t_lo) op |= 1ull << (int)(l - rowbase);
            }
            if (op) atomicOr((unsigned long long*)&sm.OPN[d][r], (unsigned long long)op);
        }
    }
    __syncthreads();

    // 3) outgoing open links (far faces) -> crossing bits; x-runs -> first
    //    parents; E and M of the incoming configuration
    {
        uint32_t* xb = R.xbits + (size_t)t * C::XW;
        for (int w = tid; w < C::XW; w += kBlock) {
            uint32_t bits = 0;
            if (w < C::W0) {                       // face x = wx-1: bit ly + TY*lz
                for (int b = 0; b < 32; ++b) {
                    const int fb = w * 32 + b;
                    if (fb >= C::F0) break;
                    const int ly = fb % C::TY, lz = fb / C::TY;
                    if (ly < g.wy && lz < g.wz) bits |= (uint32_t)((sm.OPN[0][fb] >> (g.wx - 1)) & 1ull) << b;
                }
            } else if (w < C::W0 + C::W1) {        // face y = wy-1: bit x + TX*lz
                const int fb0 = (w - C::W0) * 32;
                const int lz = fb0 / C::TX, x0 = fb0 % C::TX;
                if (lz < g.wz) bits = (uint32_t)(sm.OPN[1][(g.wy - 1) + C::TY * lz] >> x0);
            } else {                               // face z = wz-1: bit x + TX*ly
                const int fb0 = (w - C::W0 - C::W1) * 32;
                const int ly = fb0 / C::TX, x0 = fb0 % C::TX;
                if (ly < g.wy) bits = (uint32_t)(sm.OPN[C::D - 1][ly + C::TY * (g.wz - 1)] >> x0);
            }
            xb[w] = bits;
        }
        const uint64_t inside = low_bits(g.wx - 1);   // x-bonds whose both ends are in the tile
#pragma unroll 4
        for (int i = 0; i < C::SITEIT; ++i) {
            const int k = tid + kBlock * i;
            const int x = k % C::TX, r = k / C::TX;
            const int ly = r % C::TY, lz = r / C::TY;
            int p = k;
            if (x < g.wx && ly < g.wy && lz < g.wz) {
                const uint64_t run = sm.OPN[0][r] & inside;
                const uint64_t m = ~run & low_bits(x);            // closed x-bonds left of x
                const int start = m ? 64 - __clzll((long long)m) : 0;
                p = k - x + start;
                if (x == 0) sm.RR[r] = run;
            } else if (x == 0) {
                sm.RR[r] = 0;
            }
            sm.par[k] = p;
        }
        if (measure) {
            int e = 0, m = 0;
            for (int r = tid; r < C::NR; r += kBlock) {
                const int ly = r % C::TY, lz = r / C::TY;
                if (ly >= g.wy || lz >= g.wz) continue;
                const int hr = ly + (C::TY + 1) * lz;
                m += 2 * __popcll(sm.S[hr]) - g.wx;
#pragma unroll
                for (int d = 0; d < C::D; ++d) e += 2 * __popcll(eq_mask<C>(sm, ly, lz, d, g.wx)) - g.wx;
            }
            e_acc += e;
            m_acc += m;
        }
    }
    __syncthreads();

    // 4) unions across rows (y, z links inside the tile).  A link whose left
    //    neighbour link joins the same two x-runs is implied and skipped.
#pragma unroll 1
    for (int i = 0; i < C::SITEIT; ++i) {
        const int k = tid + kBlock * i;
        const int x = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        if (x >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        if (ly < g.wy - 1 && ((sm.OPN[1][r] >> x) & 1ull)) {
            const bool implied = x > 0 && (((sm.RR[r] & sm.OPN[1][r] & sm.RR[r + 1]) >> (x - 1)) & 1ull);
            if (!implied) lds_unite(sm.par, k, k + C::TX);
        }
        if (C::D == 3 && lz < g.wz - 1 && ((sm.OPN[C::D - 1][r] >> x) & 1ull)) {
            const bool implied = x > 0 && (((sm.RR[r] & sm.OPN[C::D - 1][r] & sm.RR[r + C::TY]) >> (x - 1)) & 1ull);
            if (!implied) lds_unite(sm.par, k, k + C::TX * C::TY);
        }
    }
    __syncthreads();
    // compress: one store per site, of its root.  Path halving here would race:
    // a halving store can put an intermediate ancestor back over a root that
    // another thread has just written.
    for (int k = tid; k < C::TS; k += kBlock) {
        const int root = lds_root(sm.par, k);
        lds_store(&sm.par[k], root);
    }
    __syncthreads();

    // 5) border clusters: touching a near face, or leaving through a far face
#pragma unroll 2
    for (int i = 0; i < C::SITEIT; ++i) {
        const int k = tid + kBlock * i;
        const int x = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        if (x >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        bool b = x == 0 || ly == 0 || (C::D == 3 && lz == 0);
        b = b || (x == g.wx - 1 && ((sm.OPN[0][r] >> x) & 1ull)) || (ly == g.wy - 1 && ((sm.OPN[1][r] >> x) & 1ull));
        if (C::D == 3) b = b || (lz == g.wz - 1 && ((sm.OPN[C::D - 1][r] >> x) & 1ull));
        if (b) sm.flag[sm.par[k]] = 1;
    }
    __syncthreads();

    // 6) tile-local labels; border roots start their own global tree
#pragma unroll 4
    for (int i = 0; i < C::SITEIT; ++i) {
        const int k = tid + kBlock * i;
        const int x = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        if (x >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        const int root = sm.par[k];
        const uint32_t fl = sm.flag[root] ? kBorderFlag : 0u;
        const uint32_t gi = (uint32_t)(g.x0 + x) + (uint32_t)L * ((uint32_t)(g.y0 + ly) + (uint32_t)L * (uint32_t)(g.z0 + lz));
        R.lab16[gi] = (uint16_t)((uint32_t)root | fl);
        if (root == k && fl) R.par[gi] = (int32_t)gi;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// K2: border merge over the tile's outgoing open links + flip table share.
// --------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void face_site(const TileGeo& g, int d, int fb, int& lx, int& ly, int& lz)
{
    if (d == 0) {
        lx = g.wx - 1;
        ly = fb % C::TY;
        lz = fb / C::TY;
    } else if (d == 1) {
        lx = fb % C::TX;
        ly = g.wy - 1;
        lz = fb / C::TX;
    } else {
        lx = fb % C::TX;
        ly = fb / C::TX;
        lz = g.wz - 1;
    }
}

template <class C>
__device__ void k2_tile(const SwRep& R, int t, uint32_t s)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const int L = R.L;
    const uint32_t* xb = R.xbits + (size_t)t * C::XW;
    constexpr int FT = C::F0 + C::F1 + C::F2;
    for (int it = tid; it < FT; it += kBlock) {
        int d, fb, wbase;
        if (it < C::F0) {
            d = 0;
            fb = it;
            wbase = 0;
        } else if (it < C::F0 + C::F1) {
            d = 1;
            fb = it - C::F0;
            wbase = C::W0;
        } else {
            d = 2;
            fb = it - C::F0 - C::F1;
            wbase = C::W0 + C::W1;
        }
        if (!((xb[wbase + (fb >> 5)] >> (fb & 31)) & 1u)) continue;
        int lx, ly, lz;
        face_site<C>(g, d, fb, lx, ly, lz);
        const int ax = g.x0 + lx, ay = g.y0 + ly, az = g.z0 + lz;
        const int bx = (d == 0) ? ((ax + 1 == L) ? 0 : ax + 1) : ax;
        const int by = (d == 1) ? ((ay + 1 == L) ? 0 : ay + 1) : ay;
        const int bz = (d == 2) ? ((az + 1 == L) ? 0 : az + 1) : az;
        const uint32_t ga = (uint32_t)ax + (uint32_t)L * ((uint32_t)ay + (uint32_t)L * (uint32_t)az);
        const uint32_t gb = (uint32_t)bx + (uint32_t)L * ((uint32_t)by + (uint32_t)L * (uint32_t)bz);
        const uint32_t la = R.lab16[ga], lb = R.lab16[gb];
        // the previous link along the face (first in-face axis) joining the
        // same two tile-local clusters makes this union redundant
        const int first = (d == 0) ? ly : lx;
        if (first > 0) {
            const int pfb = fb - 1;
            if ((xb[wbase + (pfb >> 5)] >> (pfb & 31)) & 1u) {
                const uint32_t step = (d == 0) ? (uint32_t)L : 1u;
                const uint32_t pa = ga - step;
                uint32_t pb;
                if (d == 0) pb = gb - (uint32_t)L;
                else pb = gb - 1u;
                if (R.lab16[pa] == la && R.lab16[pb] == lb) continue;
            }
        }
        const uint32_t ra = tile_root_of<C>(R, ga, la);
        const uint32_t rb = tile_root_of<C>(R, gb, lb);
        if (ra == 0xFFFFFFFFu || rb == 0xFFFFFFFFu) continue;
        g_unite(R, R.par, (int)ra, (int)rb);
    }
    // flip bits of this sweep: table word 4b + w is word w of Philox(b, 0, s, FLIP)
    const uint32_t nblk = (R.N + 127u) / 128u;
    const uint32_t b0 = (uint32_t)(((uint64_t)t * nblk) / (uint32_t)R.ntiles);
    const uint32_t b1 = (uint32_t)(((uint64_t)(t + 1) * nblk) / (uint32_t)R.ntiles);
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
    for (uint32_t b = b0 + (uint32_t)tid; b < b1; b += kBlock) {
        const U4 r = philox10(b, 0u, s, kTagFlip, k0, k1);
        uint4 v;
        v.x = r.x;
        v.y = r.y;
        v.z = r.z;
        v.w = r.w;
        reinterpret_cast<uint4*>(R.fliptab)[b] = v;
    }
}

// --------------------------------------------------------------------------
// K3: cluster flip.  Each distinct tile-local root is resolved once (global
// chase for border roots, flip bit from the table); sites then read their
// root's result from LDS.  Optionally marks percolation coverage (PCC).
// --------------------------------------------------------------------------
template <class C>
struct K3Smem {
    uint32_t res[C::TS];   // (cluster root << 1) | new-spin bit, per tile-local root
    uint8_t need[C::TS];   // 0: unused, 1: interior root, 2: border root
};

template <class C>
__device__ void k3_tile(const SwRep& R, int t, uint32_t s, K3Smem<C>& sm)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t L = (uint32_t)R.L;
    for (int k = tid; k < C::TS; k += kBlock) sm.need[k] = 0;
    __syncthreads();
    uint16_t v[C::SITEIT];
#pragma unroll
    for (int i = 0; i < C::SITEIT; ++i) {
        const int k = tid + kBlock * i;
        const int x = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        v[i] = 0xFFFFu;
        if (x >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        const uint32_t gi = (uint32_t)(g.x0 + x) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
        v[i] = R.lab16[gi];
        if ((uint32_t)(v[i] & 0x7FFFu) > (uint32_t)k) {   // a tile root precedes its sites
            flag_error(R, ERR_TILE_LABEL);
            v[i] = 0xFFFFu;
        }
    }
#pragma unroll
    for (int i = 0; i < C::SITEIT; ++i)
        if (v[i] != 0xFFFFu) sm.need[v[i] & 0x7FFFu] = (v[i] & kBorderFlag) ? 2 : 1;
    __syncthreads();
    for (int k = tid; k < C::TS; k += kBlock) {
        const uint8_t nd = sm.need[k];
        if (!nd) continue;
        uint32_t r = local_to_global<C>((uint32_t)k, g.x0, g.y0, g.z0, (int)L);
        if (nd == 2) r = ro_find(R, r);
        const uint32_t bit = (R.fliptab[r >> 5] >> (r & 31u)) & 1u;
        sm.res[k] = (r << 1) | bit;
    }
    __syncthreads();
    const bool pcc = (R.flags & FLAG_PCC) != 0;
    const uint64_t tag = (uint64_t)(s + 1u) << 32;
    const uint32_t bw = (L + 31u) / 32u;               // bitmap words per candidate
    const uint32_t nslots = (C::D == 3) ? L * L : L;   // candidates per axis
#pragma unroll
    for (int i = 0; i < C::SITEIT; ++i) {
        if (v[i] == 0xFFFFu) continue;
        const int k = tid + kBlock * i;
        const int x = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        const uint32_t gi = (uint32_t)(g.x0 + x) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
        const uint32_t q = sm.res[v[i] & 0x7FFFu];
        const uint32_t root = q >> 1;
        R.spins[gi] = (q & 1u) ? (int8_t)1 : (int8_t)-1;
        if (R.lab32) R.lab32[gi] = (int32_t)root;
        if (pcc) {
            const uint32_t crd[3] = {(uint32_t)(g.x0 + x), (uint32_t)(g.y0 + ly), (uint32_t)(g.z0 + lz)};
#pragma unroll
            for (int a = 0; a < C::D; ++a) {
                const uint64_t c = R.cand[(size_t)a * R.N + root];
                if ((c & 0xFFFFFFFF00000000ull) != tag) continue;
                const uint32_t slot = ~(uint32_t)c;
                if (slot >= nslots) {
                    flag_error(R, ERR_SLOT);
                    continue;
                }
                uint32_t* bm = R.bmp + ((size_t)a * nslots + slot) * bw;
                atomicOr(&bm[crd[a] >> 5], 1u << (crd[a] & 31u));
            }
        }
    }
    __syncthreads();
}

// PCC: every cluster that covers all L coordinates along axis a must meet the
// hyperplane x_a = 0, so the clusters of that hyperplane are the candidates.
// Each gets a slot (the smallest in-plane position where it meets the plane).
template <class C>
__device__ void k_cand_tile(const SwRep& R, int t, uint32_t s)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t L = (uint32_t)R.L;
    const uint64_t tag = (uint64_t)(s + 1u) << 32;
    for (int a = 0; a < C::D; ++a) {
        const int o = (a == 0) ? g.x0 : (a == 1) ? g.y0 : g.z0;
        if (o != 0) continue;                          // tile does not touch x_a = 0
        // sites of the tile with coordinate a == 0: the face spanned by the other axes
        const int fu = (a == 0) ? g.wy : g.wx;
        const int fv = (C::D == 3) ? ((a == 2) ? g.wy : g.wz) : 1;
        for (int k = tid; k < fu * fv; k += kBlock) {
            const int u = k % fu, w = k / fu;
            int x = g.x0, y = g.y0, z = g.z0;
            if (a == 0) {
                y += u;
                z += w;
            } else if (a == 1) {
                x += u;
                z += w;
            } else {
                x += u;
                y += w;
            }
            const uint32_t gi = (uint32_t)x + L * ((uint32_t)y + L * (uint32_t)z);
            const uint32_t v = R.lab16[gi];
            uint32_t r = tile_root_of<C>(R, gi, v);
            if (r == 0xFFFFFFFFu) continue;
            if (v & kBorderFlag) r = ro_find(R, r);
            // in-plane position
            uint32_t slot;
            if (C::D == 2) slot = (a == 0) ? (uint32_t)y : (uint32_t)x;
            else slot = (a == 0) ? (uint32_t)y + L * (uint32_t)z : (a == 1) ? (uint32_t)x + L * (uint32_t)z : (uint32_t)x + L * (uint32_t)y;
            atomicMax((unsigned long long*)&R.cand[(size_t)a * R.N + r], (unsigned long long)(tag | (uint64_t)(~slot)));
        }
    }
}

}  // namespace sw
