// sw_device.hpp -- device-side data layout and the per-tile phases of one
// Swendsen-Wang sweep (Lin & Zheng, Sec. I steps 1-3) on gfx950.
//
// A replica's lattice is cut into tiles of TX x TY (x TZ) sites.  One sweep is
//   K1  per tile: load spins (+ the far halo), draw the bonds of the tile's own
//       links from Philox, label the tile's clusters by union-find in LDS, write
//       a 16-bit tile-local label per site and the bits of the tile's open
//       links that leave it (the tile plays the part of a domain in Sec. II).
//   K2  per tile: join, in a global union-find over tile-local roots, the two
//       ends of every open link that leaves the tile (the border
//       reconciliation of Sec. II; one pass instead of the master's second
//       labelling or the iterated neighbour exchange), and write this sweep's
//       flip-bit table.
//   K3  per tile: resolve every site's cluster root (= the smallest site index
//       of the cluster, the label identity that Sec. II.B converges to) and
//       give the site the cluster's new spin (Sec. I step 3).
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
    uint32_t limit;             // batched engine: never run past this sweep
    uint32_t measured;          // series entries complete (E,M after sweep k, k < measured)
    uint32_t series_cap;        // entries the series buffer holds
    uint32_t trace_cap;         // entries the PCC trace buffers hold
    int32_t active;             // batched engine: replica takes part
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
};

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
    static constexpr int HX = TX + 1, HY = TY + 1, HZ = (D == 3) ? TZ + 1 : 1;
    static constexpr int HS = HX * HY * HZ;
    static constexpr int F0 = TY * TZ, F1 = TX * TZ, F2 = (D == 3) ? TX * TY : 0;
    static constexpr int W0 = (F0 + 31) / 32, W1 = (F1 + 31) / 32, W2 = (F2 + 31) / 32;
    static constexpr int XW = W0 + W1 + W2;
    static constexpr int NB = TX / 16;        // Philox bond blocks per aligned row
    static_assert(TX % 16 == 0, "tile rows hold whole 16-link bond blocks");
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
    return local_to_global<C>(v & 0x7FFFu, x0, y0, z0, (int)L);
}

// --------------------------------------------------------------------------
// Union-find primitives.  Parents only ever point to smaller indices of the
// same cluster, so the root of a cluster is its smallest member.
// --------------------------------------------------------------------------
__device__ __forceinline__ int lds_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(int* par, int x)
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

// find with path halving; safe under concurrent unions because every store
// writes an ancestor of the node it updates
__device__ __forceinline__ int g_find(int* par, int x)
{
    while (true) {
        const int p = g_load(&par[x]);
        if (p == x) return x;
        const int gp = g_load(&par[p]);
        if (gp == p) return p;
        g_store(&par[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void g_unite(int* par, int a, int b)
{
    while (true) {
        a = g_find(par, a);
        b = g_find(par, b);
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
__device__ __forceinline__ uint32_t ro_find(const int32_t* par, uint32_t x)
{
    int p = par[x];
    while ((uint32_t)p != x) {
        x = (uint32_t)p;
        p = par[x];
    }
    return x;
}

// --------------------------------------------------------------------------
// K1: bonds + tile labelling.
// --------------------------------------------------------------------------
template <class C>
struct K1Smem {
    int32_t par[C::TS];
    uint8_t bnd[C::D][C::TS];
    uint8_t flag[C::TS];
    int8_t sp[C::HS];
};

template <class C>
__device__ void k1_tile(const SwRep& R, int t, uint32_t s, uint64_t thr, K1Smem<C>& sm, bool measure,
                        int64_t& e_acc, int64_t& m_acc)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const int L = R.L;
    const uint32_t N = R.N;
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);

    // 1) spins of the tile and of the far halo (the +x, +y, +z neighbours)
    for (int k = tid; k < C::HS; k += kBlock) {
        const int hx = k % C::HX;
        const int hy = (k / C::HX) % C::HY;
        const int hz = k / (C::HX * C::HY);
        int8_t v = 0;
        const bool in = hx <= g.wx && hy <= g.wy && (C::D == 2 || hz <= g.wz);
        const int nh = (hx == g.wx) + (hy == g.wy) + ((C::D == 3) && (hz == g.wz));
        if (in && nh <= 1) {
            int gx = g.x0 + hx;
            int gy = g.y0 + hy;
            int gz = g.z0 + hz;
            if (gx == L) gx = 0;
            if (gy == L) gy = 0;
            if (C::D == 3 && gz == L) gz = 0;
            const uint32_t gi = (uint32_t)gx + (uint32_t)L * ((uint32_t)gy + (uint32_t)L * (uint32_t)gz);
            v = R.spins[gi];
        }
        sm.sp[k] = v;
    }
    for (int k = tid; k < C::TS; k += kBlock) {
        sm.par[k] = k;
        sm.flag[k] = 0;
    }
    __syncthreads();

    // 2) bonds of the tile's own links (i, d), d < D, from 16-link Philox blocks
    const uint32_t t_hi = (uint32_t)(thr >> 24);
    const uint32_t t_lo = (uint32_t)(thr & 0xFFFFFFu);
    const int nslot = (L % 16 == 0) ? C::NB : C::NB + 1;
    constexpr int rows = C::TY * C::TZ;
    const int nitems = C::D * rows * nslot;
    for (int it = tid; it < nitems; it += kBlock) {
        const int j = it % nslot;
        const int rr = (it / nslot) % rows;
        const int d = it / (nslot * rows);
        const int ly = rr % C::TY;
        const int lz = rr / C::TY;
        if (ly >= g.wy || lz >= g.wz) continue;
        const uint32_t rowbase =
            (uint32_t)d * N + (uint32_t)g.x0 + (uint32_t)L * ((uint32_t)(g.y0 + ly) + (uint32_t)L * (uint32_t)(g.z0 + lz));
        const uint32_t blk = (rowbase >> 4) + (uint32_t)j;
        const uint32_t lo = max(blk * 16u, rowbase);
        const uint32_t hi = min(blk * 16u + 16u, rowbase + (uint32_t)g.wx);
        if (lo >= hi) continue;
        const U4 r = philox10(blk, 0u, s, kTagBond, k0, k1);
        const int sbase = C::HX * (ly + C::HY * lz);
        const int nstep = (d == 0) ? 1 : (d == 1) ? C::HX : C::HX * C::HY;
        uint32_t opens = 0, ties = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t l = blk * 16u + (uint32_t)k;
            if (l < lo || l >= hi) continue;
            const uint32_t word = (k < 4) ? r.x : (k < 8) ? r.y : (k < 12) ? r.z : r.w;
            const uint32_t a = (word >> (8 * (k & 3))) & 0xFFu;
            const int si = sbase + (int)(l - rowbase);
            const bool eq = sm.sp[si] == sm.sp[si + nstep];
            if (eq && a < t_hi) opens |= 1u << k;
            if (eq && a == t_hi) ties |= 1u << k;
        }
        while (ties) {
            const int k = __ffs(ties) - 1;
            ties &= ties - 1u;
            const uint32_t l = blk * 16u + (uint32_t)k;
            const U4 q = philox10(l >> 2, 0u, s, kTagRefine, k0, k1);
            if ((pick(q, l & 3u) & 0xFFFFFFu) < t_lo) opens |= 1u << k;
        }
        const int lbase = C::TX * (ly + C::TY * lz);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t l = blk * 16u + (uint32_t)k;
            if (l < lo || l >= hi) continue;
            sm.bnd[d][lbase + (int)(l - rowbase)] = (uint8_t)((opens >> k) & 1u);
        }
    }
    __syncthreads();

    // 3) bits of the open links that leave the tile through its far faces
    uint32_t* xb = R.xbits + (size_t)t * C::XW;
    for (int w = tid; w < C::XW; w += kBlock) {
        int d, wo;
        if (w < C::W0) {
            d = 0;
            wo = w;
        } else if (w < C::W0 + C::W1) {
            d = 1;
            wo = w - C::W0;
        } else {
            d = 2;
            wo = w - C::W0 - C::W1;
        }
        const int F = (d == 0) ? C::F0 : (d == 1) ? C::F1 : C::F2;
        uint32_t bits = 0;
        for (int b = 0; b < 32; ++b) {
            const int fb = wo * 32 + b;
            if (fb >= F) break;
            int lx, ly, lz;
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
            if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
            bits |= (uint32_t)sm.bnd[d][lx + C::TX * (ly + C::TY * lz)] << b;
        }
        xb[w] = bits;
    }

    // 4) energy and magnetisation of the incoming configuration
    if (measure) {
        int e = 0, m = 0;
        for (int k = tid; k < C::TS; k += kBlock) {
            const int lx = k % C::TX, ly = (k / C::TX) % C::TY, lz = k / (C::TX * C::TY);
            if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
            const int si = lx + C::HX * (ly + C::HY * lz);
            const int sv = sm.sp[si];
            int nb = sm.sp[si + 1] + sm.sp[si + C::HX];
            if (C::D == 3) nb += sm.sp[si + C::HX * C::HY];
            m += sv;
            e += sv * nb;
        }
        e_acc += e;
        m_acc += m;
    }

    // 5) union-find over the open links inside the tile
    for (int k = tid; k < C::TS; k += kBlock) {
        const int lx = k % C::TX, ly = (k / C::TX) % C::TY, lz = k / (C::TX * C::TY);
        if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        if (lx < g.wx - 1 && sm.bnd[0][k]) lds_unite(sm.par, k, k + 1);
        if (ly < g.wy - 1 && sm.bnd[1][k]) lds_unite(sm.par, k, k + C::TX);
        if (C::D == 3 && lz < g.wz - 1 && sm.bnd[C::D - 1][k]) lds_unite(sm.par, k, k + C::TX * C::TY);
    }
    __syncthreads();
    for (int k = tid; k < C::TS; k += kBlock) sm.par[k] = lds_find(sm.par, k);
    __syncthreads();

    // 6) border clusters: touching a near face, or leaving through a far face
    for (int k = tid; k < C::TS; k += kBlock) {
        const int lx = k % C::TX, ly = (k / C::TX) % C::TY, lz = k / (C::TX * C::TY);
        if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        bool b = lx == 0 || ly == 0 || (C::D == 3 && lz == 0);
        b = b || (lx == g.wx - 1 && sm.bnd[0][k]) || (ly == g.wy - 1 && sm.bnd[1][k]);
        if (C::D == 3) b = b || (lz == g.wz - 1 && sm.bnd[C::D - 1][k]);
        if (b) sm.flag[sm.par[k]] = 1;
    }
    __syncthreads();

    // 7) tile-local labels; border roots start their own global tree
    for (int k = tid; k < C::TS; k += kBlock) {
        const int lx = k % C::TX, ly = (k / C::TX) % C::TY, lz = k / (C::TX * C::TY);
        if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        const int root = sm.par[k];
        const uint32_t fl = sm.flag[root] ? kBorderFlag : 0u;
        const uint32_t gi = (uint32_t)(g.x0 + lx) + (uint32_t)L * ((uint32_t)(g.y0 + ly) + (uint32_t)L * (uint32_t)(g.z0 + lz));
        R.lab16[gi] = (uint16_t)((uint32_t)root | fl);
        if (root == k && fl) R.par[gi] = (int32_t)gi;
    }
    __syncthreads();
}

// --------------------------------------------------------------------------
// K2: border merge over the tile's outgoing open links + flip table share.
// --------------------------------------------------------------------------
template <class C>
__device__ void k2_tile(const SwRep& R, int t, uint32_t s)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const int L = R.L;
    const uint32_t* xb = R.xbits + (size_t)t * C::XW;
    constexpr int FT = C::F0 + C::F1 + C::F2;
    for (int it = tid; it < FT; it += kBlock) {
        int d, fb, w;
        if (it < C::F0) {
            d = 0;
            fb = it;
            w = fb >> 5;
        } else if (it < C::F0 + C::F1) {
            d = 1;
            fb = it - C::F0;
            w = C::W0 + (fb >> 5);
        } else {
            d = 2;
            fb = it - C::F0 - C::F1;
            w = C::W0 + C::W1 + (fb >> 5);
        }
        if (!((xb[w] >> (fb & 31)) & 1u)) continue;
        int lx, ly, lz;
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
        const int ax = g.x0 + lx, ay = g.y0 + ly, az = g.z0 + lz;
        int bx = ax, by = ay, bz = az;
        if (d == 0) bx = (ax + 1 == L) ? 0 : ax + 1;
        if (d == 1) by = (ay + 1 == L) ? 0 : ay + 1;
        if (d == 2) bz = (az + 1 == L) ? 0 : az + 1;
        const uint32_t ga = (uint32_t)ax + (uint32_t)L * ((uint32_t)ay + (uint32_t)L * (uint32_t)az);
        const uint32_t gb = (uint32_t)bx + (uint32_t)L * ((uint32_t)by + (uint32_t)L * (uint32_t)bz);
        const uint32_t ra = tile_root_of<C>(R, ga, R.lab16[ga]);
        const uint32_t rb = tile_root_of<C>(R, gb, R.lab16[gb]);
        g_unite(R.par, (int)ra, (int)rb);
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
// K3: cluster flip.  Optionally marks percolation coverage (PCC).
// --------------------------------------------------------------------------
template <class C>
__device__ void k3_tile(const SwRep& R, int t, uint32_t s)
{
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t L = (uint32_t)R.L;
    const bool pcc = (R.flags & FLAG_PCC) != 0;
    const uint64_t tag = (uint64_t)(s + 1u) << 32;
    const uint32_t bw = (L + 31u) / 32u;               // bitmap words per candidate
    const uint32_t nslots = (C::D == 3) ? L * L : L;   // candidates per axis
    for (int k = tid; k < C::TS; k += kBlock) {
        const int lx = k % C::TX, ly = (k / C::TX) % C::TY, lz = k / (C::TX * C::TY);
        if (lx >= g.wx || ly >= g.wy || lz >= g.wz) continue;
        const uint32_t gi = (uint32_t)(g.x0 + lx) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
        const uint32_t v = R.lab16[gi];
        uint32_t r = local_to_global<C>(v & 0x7FFFu, g.x0, g.y0, g.z0, (int)L);
        if (v & kBorderFlag) r = ro_find(R.par, r);
        const uint32_t bit = (R.fliptab[r >> 5] >> (r & 31u)) & 1u;
        R.spins[gi] = bit ? (int8_t)1 : (int8_t)-1;
        if (R.lab32) R.lab32[gi] = (int32_t)r;
        if (pcc) {
            const uint32_t crd[3] = {(uint32_t)(g.x0 + lx), (uint32_t)(g.y0 + ly), (uint32_t)(g.z0 + lz)};
#pragma unroll
            for (int a = 0; a < C::D; ++a) {
                const uint64_t c = R.cand[(size_t)a * R.N + r];
                if ((c & 0xFFFFFFFF00000000ull) != tag) continue;
                const uint32_t slot = ~(uint32_t)c;
                uint32_t* bm = R.bmp + ((size_t)a * nslots + slot) * bw;
                atomicOr(&bm[crd[a] >> 5], 1u << (crd[a] & 31u));
            }
        }
    }
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
            if (v & kBorderFlag) r = ro_find(R.par, r);
            // in-plane position
            uint32_t slot;
            if (C::D == 2) slot = (a == 0) ? (uint32_t)y : (uint32_t)x;
            else slot = (a == 0) ? (uint32_t)y + L * (uint32_t)z : (a == 1) ? (uint32_t)x + L * (uint32_t)z : (uint32_t)x + L * (uint32_t)y;
            atomicMax((unsigned long long*)&R.cand[(size_t)a * R.N + r], (unsigned long long)(tag | (uint64_t)(~slot)));
        }
    }
}

}  // namespace sw
