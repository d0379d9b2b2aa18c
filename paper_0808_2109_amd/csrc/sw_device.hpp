// sw_device.hpp -- device-side data layout and the per-tile phases of one
// Swendsen-Wang sweep (Lin & Zheng, Sec. I steps 1-3) on gfx950.
//
// A replica's lattice is cut into tiles of TX x TY (x TZ) sites, TX = 32 or
// 64, so that every wave64 covers whole tile rows.  One sweep is
//   K1  per tile: load the spins (+ the far halo) as one bit mask per row,
//       draw the bonds of the tile's own links from Philox as bit masks, label
//       the tile's clusters in LDS (runs along x from the bond masks, a
//       union-find over the runs of neighbouring rows), write a 16-bit
//       tile-local label per site, the bits of the tile's open links that
//       leave it, its border roots (tile roots of clusters that reach its
//       faces), each with a slot of the border merge's union-find, and for
//       every face site the slot rank of its tile root.  The tile plays the
//       part of a domain of Sec. II.
//   K2  per far-face site: join, in the global union-find over the border
//       roots' slots, the two ends of every open link that leaves a tile (the
//       border reconciliation of Sec. II, in one pass instead of the master's
//       second labelling or the iterated neighbour exchange).
//   K3a per tile: find the cluster root of each of the tile's border roots
//       (the smallest site index of the cluster: the label identity that the
//       min-label rule of Sec. II.B converges to) and that cluster's flip bit.
//   K3b per tile: give every site its cluster's new spin (Sec. I step 3).
// plus the percolation tests and p feedback of Sec. III (extension rule,
// open-box spanning, topological rule).
//
// Every union hooks the larger root under the smaller one, so the final roots
// do not depend on the order of unions, the tile shape or the schedule: the
// result is bit-identical to a sequential labelling.
#pragma once
#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
#ifndef SW_K3_THREADS
#define SW_K3_THREADS 256
#endif
constexpr int kK3Block = SW_K3_THREADS;  // threads per K3 workgroup
constexpr uint32_t kTagInit = 0, kTagBond = 1, kTagRefine = 2, kTagFlip = 3;

enum : uint32_t { FLAG_SERIES = 1u, FLAG_KEEP = 2u, FLAG_PCC = 4u, FLAG_BITPACK = 8u, FLAG_OPEN = 16u, FLAG_WIND = 32u };

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
    int32_t fbw;                // words of a per-tile site bitmap (TS / 32)
    int32_t ft;                 // face sites per face set of a tile (F0 + F1 + F2)
    uint32_t flags;
    uint64_t seed;
    uint64_t thr;               // threshold of the next sweep (<= 2^32)
    double p;                   // bond probability of the next sweep
    double dp0;                 // PCC step at sweep 0
    uint32_t halve_every;       // PCC: dp halves every this many sweeps
    uint32_t sweep;             // sweeps done
    uint32_t limit;             // batched mode: never run past this sweep
    uint32_t measured;          // series entries complete (E,M after sweep k, k < measured)
    uint32_t first;             // first sweep of the records: series row j and PCC trace entry j
                                // belong to sweep first + j (the resume point of the last set_spins)
    uint32_t series_cap;        // entries the series buffer holds
    uint32_t trace_cap;         // entries the PCC trace buffers hold
    int32_t active;             // batched mode: replica takes part
    int8_t* spins;              // N int8 +1/-1; with FLAG_BITPACK ceil(N/32) uint32 words instead,
                                // site i up iff bit i%32 of word i/32 is set
    uint16_t* lab16;            // N tile-local labels (tile-local index of the cluster's tile root),
                                // allocated for N rounded up to a multiple of 4
    int32_t* par;               // FLAG_KEEP: N entries, the cluster root of every border root (K3a -> K3b)
    uint64_t* dpar;             // the border merge's union-find over the border roots, which
                                // hold the slots [t * 2ft, t * 2ft + nb_t) of their tile t in
                                // rank order; an entry is (parent's site << 32 | parent's slot)
                                // and a root's names itself (not with FLAG_WIND)
    uint64_t* par64;            // FLAG_WIND: N entries (parent | sheet offsets << 32) of the border
                                // merge's union-find, which then takes the place of dpar
    uint16_t* fpre;             // PCC (not FLAG_WIND): ntiles * fbw, border roots before each
                                // word of the tile's border bitmap (the rank of a border root)
    uint32_t nslots;            // ntiles * 2 * ft: slots of dpar
    int32_t* lab32;             // N final labels (FLAG_KEEP), else null
    uint32_t* xbits;            // ntiles * xwords crossing-link bits
    uint32_t* fbits;            // ntiles * fbw: border roots of each tile (bit per tile-local site)
    uint16_t* face;             // ntiles * 2 * ft: near, then far face sites: the rank of the site's
                                // tile root among the tile's border roots (FLAG_WIND: the tile-local
                                // label itself)
    uint32_t* bflip;            // ntiles * fbw: flip bit of every tile-local root (K3a -> K3b)
    int64_t* series;            // 2 * series_cap
    int64_t* acc;               // 2 scratch accumulators (measure)
    uint64_t* cand;             // PCC: dim * N candidate marks (tag << 32 | ~slot)
    uint64_t* cov;              // PCC: per tile, 2 * ft entries of two words: the coverage of each
                                // border root within the tile (K1 -> K3a)
    uint32_t* bmp;              // PCC: dim * L^(dim-1) * ceil(L/32) coverage bitmaps
    int32_t* pflag;             // PCC: percolation flag of the current sweep
    int32_t* perc_trace;        // PCC: trace_cap flags
    double* p_trace;            // PCC: trace_cap values of p after each update
    int32_t* err;               // consistency-check bits (shared by a handle's replicas)
};

// consistency checks on data-dependent indices: a violation sets a bit that
// the host turns into an error instead of letting the access go out of range
enum : int { ERR_TILE_LABEL = 1, ERR_PARENT = 2, ERR_SLOT = 3, ERR_WIND_RANGE = 4, ERR_BARRIER = 5 };

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
    static constexpr int FT = F0 + F1 + F2;   // face sites per face set (x, y, z faces in turn)
    static constexpr int FBW = TS / 32;       // words of a bitmap over the tile's sites
    static constexpr int NB = TX / 16;        // Philox bond blocks per aligned row
    static_assert(TX == 32 || TX == 64, "a wave64 covers whole tile rows");
    static_assert(TS % kBlock == 0, "whole sites per thread");
    static_assert(TS % (4 * kK3Block) == 0, "whole quads of sites per K3 thread");
    static_assert(NR <= kBlock, "one thread per row for the halo column");
    static_assert(TS <= 8192, "tile-local labels fit 13 bits of the merge keys");
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
    const uint32_t lr = v;
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
// hooks with an atomic min and retries from the value it displaced.  In LDS
// (the tile labelling) the two chains of a union are walked together and its
// ends are then pointed at the joint root.
// --------------------------------------------------------------------------
__device__ __forceinline__ int lds_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Union of the sets of a and b for the tile labelling: both chains are walked
// together (one LDS round trip per step), the larger root is hooked under the
// smaller with an atomic min (from the displaced parent again when another
// thread hooked it first), and a and b then point straight at the joint root,
// which is an ancestor of both, so the store keeps every set intact.
__device__ __forceinline__ void lds_join(int* par, int a, int b)
{
    const int a0 = a, b0 = b;
    int lo;
    while (true) {
        while (true) {
            const int pa = lds_load(&par[a]);
            const int pb = lds_load(&par[b]);
            if (pa == a && pb == b) break;
            a = pa;
            b = pb;
        }
        lo = min(a, b);
        if (a == b) break;
        const int hi = max(a, b);
        const int old = atomicMin(&par[hi], lo);
        if (old == hi) break;
        a = old;
        b = lo;
    }
    if (a0 != lo) lds_store(&par[a0], lo);
    if (b0 != lo) lds_store(&par[b0], lo);
}

// the parent of x in the topological rule's union-find (the low word of its
// 64-bit entry)
__device__ __forceinline__ int gpar(const SwRep& R, uint32_t x)
{
    return (int)(uint32_t)R.par64[x];
}

// read-only find of the roots of a and b in the topological rule's
// union-find (after all unions), the two chains walked together (one round
// trip per step of the longer one)
__device__ __forceinline__ void ro_find2(const SwRep& R, uint32_t& a, uint32_t& b)
{
    int pa = gpar(R, a), pb = gpar(R, b);
    while ((uint32_t)pa != a || (uint32_t)pb != b) {
        if (pa < 0 || (uint32_t)pa > a || pb < 0 || (uint32_t)pb > b) {
            flag_error(R, ERR_PARENT);
            return;
        }
        a = (uint32_t)pa;
        b = (uint32_t)pb;
        pa = gpar(R, a);
        pb = gpar(R, b);
    }
}

// --------------------------------------------------------------------------
// The border merge's union-find over slots.  Only border roots take part in
// the merge, so each tile gives its border roots consecutive slots (rank
// order in the tile's border bitmap) and the forest lives in a dense array a
// few entries per tile long, instead of at scattered site indices.  An entry
// holds the parent's site index in its high word and the parent's slot in
// its low word; a root's entry names itself.  Hook-to-min on the site index
// (the high word decides a 64-bit atomic min) keeps the smallest site of a
// cluster as its root, the canonical label.
// --------------------------------------------------------------------------
constexpr uint64_t kBrokenEntry = ~0ull;

__device__ __forceinline__ uint64_t pack_node(uint32_t site, uint32_t slot)
{
    return ((uint64_t)site << 32) | (uint64_t)slot;
}

__device__ __forceinline__ uint64_t d_load(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root entry of slot s (whose site is x, or ~0u when unknown) with path
// halving; parents are checked to lie in range and to have smaller sites
__device__ __forceinline__ uint64_t d_find(const SwRep& R, uint32_t s, uint32_t x)
{
    uint64_t* D = R.dpar;
    while (true) {
        const uint64_t e = d_load(&D[s]);
        const uint32_t ps = (uint32_t)e, px = (uint32_t)(e >> 32);
        if (ps == s) return e;
        if (ps >= R.nslots || px >= x) {
            flag_error(R, ERR_PARENT);
            return kBrokenEntry;
        }
        const uint64_t f = d_load(&D[ps]);
        const uint32_t gs = (uint32_t)f, gx = (uint32_t)(f >> 32);
        if (gs == ps) return f;
        if (gs >= R.nslots || gx >= px) {
            flag_error(R, ERR_PARENT);
            return kBrokenEntry;
        }
        __hip_atomic_store(&D[s], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // s skips to its grandparent
        s = gs;
        x = gx;
    }
}

__device__ __forceinline__ void d_unite(const SwRep& R, uint32_t sa, uint32_t xa, uint32_t sb, uint32_t xb)
{
    while (true) {
        const uint64_t ra = d_find(R, sa, xa), rb = d_find(R, sb, xb);
        if (ra == kBrokenEntry || rb == kBrokenEntry || ra == rb) return;
        const uint64_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        const uint64_t old = __hip_atomic_fetch_min(&R.dpar[(uint32_t)hi], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == hi) return;
        // hi had been hooked to `old` meanwhile: join that one with lo instead
        sa = (uint32_t)old;
        xa = (uint32_t)(old >> 32);
        sb = (uint32_t)lo;
        xb = (uint32_t)(lo >> 32);
    }
}

// read-only find of the cluster root's site, for phases after all unions;
// x is the site of slot s
__device__ __forceinline__ uint32_t d_ro_find(const SwRep& R, uint32_t s, uint32_t x)
{
    uint64_t e = d_load(&R.dpar[s]);
    while ((uint32_t)e != s) {
        const uint32_t ps = (uint32_t)e, px = (uint32_t)(e >> 32);
        if (ps >= R.nslots || px >= x) {
            flag_error(R, ERR_PARENT);
            return x;
        }
        s = ps;
        x = px;
        e = d_load(&R.dpar[s]);
    }
    return (uint32_t)(e >> 32);
}

// d_ro_find of two slots, their chains walked together
__device__ __forceinline__ void d_ro_find2(const SwRep& R, uint32_t sa, uint32_t& xa, uint32_t sb, uint32_t& xb)
{
    uint64_t ea = d_load(&R.dpar[sa]), eb = d_load(&R.dpar[sb]);
    while ((uint32_t)ea != sa || (uint32_t)eb != sb) {
        const uint32_t pa = (uint32_t)ea, pb = (uint32_t)eb;
        const uint32_t qa = (uint32_t)(ea >> 32), qb = (uint32_t)(eb >> 32);
        if (pa >= R.nslots || pb >= R.nslots || (pa != sa && qa >= xa) || (pb != sb && qb >= xb)) {
            flag_error(R, ERR_PARENT);
            return;
        }
        sa = pa;
        xa = qa;
        sb = pb;
        xb = qb;
        ea = d_load(&R.dpar[sa]);
        eb = d_load(&R.dpar[sb]);
    }
    xa = (uint32_t)(ea >> 32);
    xb = (uint32_t)(eb >> 32);
}

// --------------------------------------------------------------------------
// Union-find with sheet offsets, for the topological rule of Sec. III (a
// cluster winds around the periodic box).  Every site of a tile-local
// cluster lies on one sheet of the box's unwrapped cover (no link inside a
// tile wraps), so a border root carries its cluster's sheet.  An entry holds
// the parent in its low word and, above it, the sheet of the node minus the
// sheet of its parent as three signed bytes (x, y, z).  A link that leaves
// the box's last tile along axis d wraps: it moves one sheet along d.  A link
// between two sites already in one set whose sheets disagree with the link
// closes a loop around the box: the cluster winds.  Hooks (larger root under
// the smaller, as in d_unite) are compare-and-swaps of a root's whole entry;
// path halving stores composed offsets, which stay valid because an entry
// only ever relates a node to one of its ancestors.
// --------------------------------------------------------------------------
struct Sheet {
    int v[3];
};

__device__ __forceinline__ uint64_t pack64(uint32_t parent, const Sheet& k)
{
    return (uint64_t)parent | ((uint64_t)(uint8_t)k.v[0] << 32) | ((uint64_t)(uint8_t)k.v[1] << 40) |
           ((uint64_t)(uint8_t)k.v[2] << 48);
}

__device__ __forceinline__ Sheet sheet_of(uint64_t e)
{
    return Sheet{{(int)(int8_t)(e >> 32), (int)(int8_t)(e >> 40), (int)(int8_t)(e >> 48)}};
}

__device__ __forceinline__ Sheet sheet_add(const SwRep& R, const Sheet& a, const Sheet& b)
{
    Sheet c;
    for (int d = 0; d < 3; ++d) {
        c.v[d] = a.v[d] + b.v[d];
        if (c.v[d] > 127 || c.v[d] < -127) {   // never near on a box of this size; reported, not wrapped
            flag_error(R, ERR_WIND_RANGE);
            c.v[d] = 0;
        }
    }
    return c;
}

__device__ __forceinline__ uint64_t g_load64(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of x and the sheet of x minus the sheet of the root (-1: broken entry)
__device__ __forceinline__ int g_find64(const SwRep& R, uint32_t x, Sheet& k)
{
    k = Sheet{{0, 0, 0}};
    uint64_t* par = R.par64;
    while (true) {
        const uint64_t e = g_load64(&par[x]);
        const uint32_t p = (uint32_t)e;
        if (p == x) return (int)x;
        if (p > x) {
            flag_error(R, ERR_PARENT);
            return -1;
        }
        const uint64_t f = g_load64(&par[p]);
        const uint32_t gp = (uint32_t)f;
        if (gp == p) {
            k = sheet_add(R, k, sheet_of(e));
            return (int)p;
        }
        if (gp > p) {
            flag_error(R, ERR_PARENT);
            return -1;
        }
        const Sheet kx = sheet_add(R, sheet_of(e), sheet_of(f));   // x relative to its grandparent
        __hip_atomic_store(&par[x], pack64(gp, kx), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        k = sheet_add(R, k, kx);
        x = gp;
    }
}

// union of a and b across a link that moves w sheets (sheet(b) = sheet(a) + w);
// sets the replica's percolation flag when the link closes a loop around the box
__device__ __forceinline__ void g_unite64(const SwRep& R, uint32_t a, uint32_t b, const Sheet& w)
{
    while (true) {
        Sheet ka, kb;
        const int ra = g_find64(R, a, ka), rb = g_find64(R, b, kb);
        if (ra < 0 || rb < 0) return;
        Sheet d;   // sheet(rb) - sheet(ra)
        for (int c = 0; c < 3; ++c) d.v[c] = w.v[c] - kb.v[c] + ka.v[c];
        if (ra == rb) {
            if (d.v[0] | d.v[1] | d.v[2]) atomicOr(R.pflag, 1);
            return;
        }
        uint32_t lo = (uint32_t)ra, hi = (uint32_t)rb;
        if (ra > rb) {
            lo = (uint32_t)rb;
            hi = (uint32_t)ra;
            for (int c = 0; c < 3; ++c) d.v[c] = -d.v[c];
        }
        uint64_t expect = pack64(hi, Sheet{{0, 0, 0}});
        if (__hip_atomic_compare_exchange_strong(&R.par64[hi], &expect, pack64(lo, d), __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        // hi was hooked meanwhile: start again from the two sites
    }
}

// --------------------------------------------------------------------------
// Bit tools.
// --------------------------------------------------------------------------
// Per-byte unsigned compares of x against the byte y (y4 = y * 0x01010101):
// the top bit of each byte of the result holds that byte's answer.  No borrow
// or carry crosses a byte boundary: (x | 0x80) - (y & 0x7F) >= 1 per byte.
__device__ __forceinline__ uint32_t bytes_lt(uint32_t x, uint32_t y4)
{
    const uint32_t d = (x | 0x80808080u) - (y4 & 0x7F7F7F7Fu);
    return ((~x & y4) | (~(x ^ y4) & ~d)) & 0x80808080u;
}

__device__ __forceinline__ uint32_t bytes_eq(uint32_t x, uint32_t y4)
{
    const uint32_t z = x ^ y4;
    return ~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;
}

// nonzero when some byte of v is zero (exact as a whole-word test)
__device__ __forceinline__ uint32_t has_zero_byte(uint32_t v) { return (v - 0x01010101u) & ~v & 0x80808080u; }

// top bits of the four bytes (bits 7, 15, 23, 31) -> bits 0..3
__device__ __forceinline__ uint32_t byte_msbs(uint32_t m) { return (((m >> 7) * 0x00204081u) >> 21) & 0xFu; }

__device__ __forceinline__ uint32_t nibbles4(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    return byte_msbs(a) | (byte_msbs(b) << 4) | (byte_msbs(c) << 8) | (byte_msbs(d) << 12);
}

// highest set bit of s at or below x, 0 <= x < 64 (s has bit 0 set)
__device__ __forceinline__ int start_at(uint64_t s, int x)
{
    return 63 - __clzll((long long)(s & (~0ull >> (63 - x))));
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// LDS writes of this wave become visible to its other lanes (a wave's LDS
// operations complete in order; this keeps the compiler from reordering)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// flip bit of the cluster whose canonical label is c in sweep s
__device__ __forceinline__ uint32_t flip_bit(uint32_t c, uint32_t s, uint32_t k0, uint32_t k1)
{
    const U4 q = philox10(c >> 7, 0u, s, kTagFlip, k0, k1);
    return (pick(q, (c >> 5) & 3u) >> (c & 31u)) & 1u;
}

// flip bits of the wx sites gb .. gb+wx-1 (bit x <- site gb + x)
__device__ __forceinline__ uint64_t row_flips(uint32_t gb, int wx, uint32_t s, uint32_t k0, uint32_t k1)
{
    uint64_t m = 0;
    const uint32_t w0 = gb >> 5, w1 = (gb + (uint32_t)wx - 1u) >> 5;
    uint32_t cur = 0xFFFFFFFFu;
    U4 q{0u, 0u, 0u, 0u};
    for (uint32_t w = w0; w <= w1; ++w) {
        if ((w >> 2) != cur) {
            cur = w >> 2;
            q = philox10(cur, 0u, s, kTagFlip, k0, k1);
        }
        const uint64_t word = pick(q, w & 3u);
        const int sh = (int)(w * 32u - gb);        // in [-31, 63]
        m |= (sh >= 0) ? (word << sh) : (word >> (-sh));
    }
    return m & low_bits(wx);
}

// --------------------------------------------------------------------------
// K1: bonds + tile labelling.  A tile has 64 rows (TY * TZ); each row is
// split into parts of 16 sites, one thread per part (RQ = TX / 16 threads
// per row, NT = 64 * RQ threads per tile, the RQ threads of a row adjacent in
// one wave).
//
// A row is a set of bit masks over x, which every thread of the row holds
// whole: S (spin up), OPN[d] (open bond of the link (x, d)) and SS (run
// starts).  A run is a maximal stretch of a row joined by x-bonds; its node in
// the union-find is its first site.  Unions only join runs of neighbouring
// rows: for each pair of rows (y or z neighbours) one union per pair of
// overlapping runs that share an open bond, made by the thread whose part
// holds the first such bond.
// --------------------------------------------------------------------------
constexpr int kRing = 128;   // per-wave union queue entries (a power of two, >= 2 x 64)

template <class C>
struct K1Cfg {
    static constexpr int RQ = C::TX / 16;      // threads per row
    static constexpr int NT = C::NR * RQ;      // threads per tile
    static_assert(C::NR == 64, "64 rows per tile");
};

// PCC coverage of the tile's border roots, indexed by rank (the number of
// border roots before it in the border bitmap): a holds the x columns the
// cluster occupies in the tile (bit lx); b the rows (2D: bit ly; 3D: bit ly
// and bit TY + lz)
template <class C, bool PCC>
struct K1Cov {
};

template <class C>
struct K1Cov<C, true> {
    static constexpr int CAP = 2 * C::FT;   // a border root has a site on a near face or a far-face link
    unsigned long long a[CAP];
    unsigned long long b[CAP];
};

template <class C, bool PCC>
struct alignas(16) K1Smem {
    int32_t par[C::TS];    // parents of the run starts (tile-local site indices)
    uint32_t FB[C::FBW];   // border flag of every tile-local root
    uint64_t S[C::NR];     // spin-up masks of the rows
    uint64_t SS[C::NR];    // run starts of the rows
    uint32_t XF[2];        // open links leaving through the far x face (bit = row)
    union {
        uint32_t ring[kBlock / 64][kRing];   // step 3: per-wave queue of pending unions
        struct {
            int32_t pre[C::FBW];             // border roots before each word of FB (their ranks)
            union {
                alignas(16) uint16_t fst[2 * C::FT];   // steps 4-4a: tile-local labels of the near, then the far face sites
                K1Cov<C, PCC> cov;                     // step 4b (PCC)
            };
        };
    };
};

// spins of 4 / 16 sites -> their up bits (a spin is up when it is positive)
__device__ __forceinline__ uint32_t up4(uint32_t w)
{
    const uint32_t nz = (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;   // byte != 0
    return byte_msbs(nz & ~w);
}

__device__ __forceinline__ uint32_t up16(uint4 v)
{
    return up4(v.x) | (up4(v.y) << 4) | (up4(v.z) << 8) | (up4(v.w) << 12);
}

// up bits of the n <= 16 sites p[0 .. n-1]; `wide` when p is 16-byte aligned and n = 16
__device__ __forceinline__ uint32_t load_part(const int8_t* p, int n, bool wide)
{
    if (wide) return up16(*reinterpret_cast<const uint4*>(p));
    uint32_t m = 0;
    for (int x = 0; x < n; ++x) m |= (uint32_t)(p[x] > 0) << x;
    return m;
}

// the n <= 32 bits from bit position pos of a packed array (reads the second
// word only when the bits cross into it, so never past the last site)
__device__ __forceinline__ uint32_t packed_bits(const uint32_t* w, uint32_t pos, int n)
{
    const uint32_t i = pos >> 5, sh = pos & 31u;
    uint32_t v = w[i] >> sh;
    if (sh + (uint32_t)n > 32u) v |= w[i + 1] << (32u - sh);
    return n >= 32 ? v : v & ((1u << n) - 1u);
}

// up bits of the n <= 16 sites from site index i, int8 or bit-packed.  A
// part that does not start on a 16-byte boundary is read as the five aligned
// words around it, cut with byte alignment, when those words lie inside the
// array (sites past the part's n are read and masked off).
__device__ __forceinline__ uint32_t load_spins(const SwRep& R, uint32_t i, int n, bool wide)
{
    if (R.flags & FLAG_BITPACK) return packed_bits(reinterpret_cast<const uint32_t*>(R.spins), i, n);
    if (!wide && (i & ~3u) + 20u <= R.N) {
        const uint32_t* w = reinterpret_cast<const uint32_t*>(R.spins + (i & ~3u));
        const uint32_t sh = i & 3u;
        const uint32_t d0 = w[0], d1 = w[1], d2 = w[2], d3 = w[3], d4 = w[4];
        const uint32_t m = up16(make_uint4(__builtin_amdgcn_alignbyte(d1, d0, sh), __builtin_amdgcn_alignbyte(d2, d1, sh),
                                           __builtin_amdgcn_alignbyte(d3, d2, sh), __builtin_amdgcn_alignbyte(d4, d3, sh)));
        return m & (uint32_t)low_bits(n);
    }
    return load_part(R.spins + i, n, wide);
}

__device__ __forceinline__ uint32_t spin_up(const SwRep& R, uint32_t i)
{
    if (R.flags & FLAG_BITPACK) return (reinterpret_cast<const uint32_t*>(R.spins)[i >> 5] >> (i & 31u)) & 1u;
    return R.spins[i] > 0;
}

// bit masks of a row's RQ parts (16 bits at 16q) -> the whole row, in every
// thread of the row
template <int RQ>
__device__ __forceinline__ uint64_t row_gather(uint32_t part, int q)
{
    uint64_t v = (uint64_t)part << (16 * q);
    if (RQ >= 2) v |= __shfl_xor(v, 1, 64);
    if (RQ >= 4) v |= __shfl_xor(v, 2, 64);
    return v;
}

// Bonds of a part of up to 16 links lbase + x whose ends are equal (eq; the
// bits of links past the part's end are clear): the bonds that the high bytes
// decide (byte a of Philox(l >> 4, 0, s, BOND) for link l is the high byte of
// its uniform), and in `ties` the equal links whose byte equals thr >> 24
// (decided by the REFINE stream; the caller draws those for all directions
// in one loop, so a wave pays about one refinement call per sweep instead of
// one per direction).  When the part does not start on a 16-link boundary
// (L not a multiple of 16) its 16 bytes are bytes o..15 of one BOND block and
// 0..o-1 of the next, o = lbase mod 16: both blocks are drawn and the window
// is cut out of their eight words.
__device__ __forceinline__ uint32_t part_bonds_coarse(uint32_t eq, uint32_t lbase, uint32_t s, uint32_t t_hi,
                                                      uint32_t k0, uint32_t k1, uint32_t& ties)
{
    ties = 0;
    if (!eq) return 0;
    if (t_hi >= 256u) return eq;                     // P = 1: every equal link is a bond
    const uint32_t y4 = t_hi * 0x01010101u;
    U4 q = philox10(lbase >> 4, 0u, s, kTagBond, k0, k1);
    const uint32_t o = lbase & 15u;
    if (o) {
        const U4 n = philox10((lbase >> 4) + 1u, 0u, s, kTagBond, k0, k1);
        const uint32_t w[8] = {q.x, q.y, q.z, q.w, n.x, n.y, n.z, n.w};
        const uint32_t j = o >> 2, sh = o & 3u;   // first word, byte offset within it
        uint32_t v[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = (j == 0) ? w[i] : (j == 1) ? w[i + 1] : (j == 2) ? w[i + 2] : w[i + 3];
        q = U4{__builtin_amdgcn_alignbyte(v[1], v[0], sh), __builtin_amdgcn_alignbyte(v[2], v[1], sh),
               __builtin_amdgcn_alignbyte(v[3], v[2], sh), __builtin_amdgcn_alignbyte(v[4], v[3], sh)};
    }
    const uint32_t bits = nibbles4(bytes_lt(q.x, y4), bytes_lt(q.y, y4), bytes_lt(q.z, y4), bytes_lt(q.w, y4)) & eq;
    if (has_zero_byte(q.x ^ y4) | has_zero_byte(q.y ^ y4) | has_zero_byte(q.z ^ y4) | has_zero_byte(q.w ^ y4))
        ties = nibbles4(bytes_eq(q.x, y4), bytes_eq(q.y, y4), bytes_eq(q.z, y4), bytes_eq(q.w, y4)) & eq;
    return bits;
}

// Threads beyond K1Cfg<C>::NT (a workgroup sized for a larger tile) take part
// in the barriers only.  With PCC the tile also records, for each border
// root, the columns and rows its cluster occupies in the tile.
template <class C, bool PCC>
__device__ void k1_tile(const SwRep& R, int t, uint32_t s, uint64_t thr, K1Smem<C, PCC>& sm, bool measure,
                        int64_t& e_acc, int64_t& m_acc)
{
    using K = K1Cfg<C>;
    constexpr int RQ = K::RQ;
    const int tid = threadIdx.x;
    const bool active = tid < K::NT;
    const int r = active ? tid / RQ : 0, q = tid % RQ;
    const int ly = r % C::TY, lz = r / C::TY;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t L = (uint32_t)R.L;
    const uint32_t N = R.N;
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
    const bool rowok = active && ly < g.wy && lz < g.wz;
    const int xp = 16 * q;                                  // first site of this thread's part
    const int np = max(0, min(16, g.wx - xp));              // sites of the part inside the tile
    const bool partok = rowok && np > 0;
    const uint64_t lbw = low_bits(g.wx);
    const bool wide = (L & 15u) == 0;                       // rows and parts start on 16-site boundaries
    const uint32_t yy = (uint32_t)(g.y0 + ly), zz = (uint32_t)(g.z0 + lz);
    const uint32_t gi0 = (uint32_t)g.x0 + L * (yy + L * zz);   // first site of the row
    const bool edgeY = ly == g.wy - 1, edgeZ = C::D == 3 && lz == g.wz - 1;

    // 1) spins: the row, the +x halo site, and for the last row in y / z of
    //    the tile the neighbour row beyond it
    uint32_t mine = partok ? load_spins(R, gi0 + (uint32_t)xp, np, wide) : 0u;
    const uint64_t S = row_gather<RQ>(mine, q);
    uint32_t hb = 0;
    if (rowok && q == RQ - 1) {
        const uint32_t hx = ((uint32_t)(g.x0 + g.wx) == L) ? 0u : (uint32_t)(g.x0 + g.wx);
        hb = spin_up(R, hx + L * (yy + L * zz));
    }
    const uint64_t HB = __shfl(hb, (threadIdx.x & 63) | (RQ - 1), 64);
    uint32_t ypart = 0, zpart = 0;
    if (partok && edgeY) {
        const uint32_t ny = (yy + 1u == L) ? 0u : yy + 1u;
        ypart = load_spins(R, (uint32_t)g.x0 + L * (ny + L * zz) + (uint32_t)xp, np, wide);
    }
    if (C::D == 3 && partok && edgeZ) {
        const uint32_t nz = (zz + 1u == L) ? 0u : zz + 1u;
        zpart = load_spins(R, (uint32_t)g.x0 + L * (yy + L * nz) + (uint32_t)xp, np, wide);
    }
    const uint64_t HY = row_gather<RQ>(ypart, q);
    const uint64_t HZ = (C::D == 3) ? row_gather<RQ>(zpart, q) : 0ull;
    if (active && q == 0) sm.S[r] = S;
    if (tid < 2) sm.XF[tid] = 0;
    for (int w = tid; w < C::FBW; w += blockDim.x) sm.FB[w] = 0;
    for (int k = 4 * tid; k < C::TS; k += 4 * (int)blockDim.x)
        *reinterpret_cast<uint4*>(&sm.par[k]) = make_uint4((uint32_t)k, (uint32_t)k + 1u, (uint32_t)k + 2u, (uint32_t)k + 3u);
    __syncthreads();

    // 2) bonds of the row's own links (x, d), each thread those of its part.
    //    With open boundaries the links that would wrap around the box do not
    //    exist (ex[d]): they never bond and are left out of E_int.
    uint64_t opn[3] = {0, 0, 0};
    {
        uint64_t eq[3] = {0, 0, 0};
        uint64_t ex[3] = {lbw, lbw, lbw};
        if (R.flags & FLAG_OPEN) {
            if ((uint32_t)(g.x0 + g.wx) == L) ex[0] &= ~(1ull << (g.wx - 1));
            if (yy == L - 1u) ex[1] = 0;
            if (C::D == 3 && zz == L - 1u) ex[2] = 0;
        }
        if (rowok) {
            eq[0] = ~(S ^ ((S >> 1) | (HB << (g.wx - 1)))) & ex[0];
            const uint64_t nbY = edgeY ? HY : sm.S[min(r + 1, C::NR - 1)];
            eq[1] = ~(S ^ nbY) & ex[1];
            if (C::D == 3) {
                const uint64_t nbZ = edgeZ ? HZ : sm.S[min(r + C::TY, C::NR - 1)];
                eq[2] = ~(S ^ nbZ) & ex[2];
            }
        }
        const uint32_t t_hi = (uint32_t)(thr >> 24);
        const uint32_t t_lo = (uint32_t)(thr & 0xFFFFFFu);
        uint32_t bits[3] = {0u, 0u, 0u};
        uint64_t ties = 0;                                   // bit 16 d + j: link (xp + j, d) needs REFINE
#pragma unroll
        for (int d = 0; d < C::D; ++d) {
            const uint32_t eqp = (uint32_t)(eq[d] >> xp) & 0xFFFFu;
            const uint32_t lbase = (uint32_t)d * N + gi0 + (uint32_t)xp;
            if (partok) {   // (a part cut short by the tile's edge has the bits past its end clear in eq)
                uint32_t td;
                bits[d] = part_bonds_coarse(eqp, lbase, s, t_hi, k0, k1, td);
                ties |= (uint64_t)td << (16 * d);
            }
        }
        while (ties) {
            const int b = __builtin_ctzll(ties);
            ties &= ties - 1ull;
            const int d = b >> 4, j = b & 15;
            const uint32_t l = (uint32_t)d * N + gi0 + (uint32_t)(xp + j);
            const U4 q2 = philox10(l >> 2, 0u, s, kTagRefine, k0, k1);
            if ((pick(q2, l & 3u) & 0xFFFFFFu) < t_lo) bits[d] |= 1u << j;
        }
#pragma unroll
        for (int d = 0; d < C::D; ++d) opn[d] = row_gather<RQ>(bits[d], q);
        if (measure && partok) {
            const uint64_t pm = low_bits(np) << xp;
            m_acc += 2 * (int)__popcll(S & pm) - np;         // __popcll is unsigned
#pragma unroll
            for (int d = 0; d < C::D; ++d) e_acc += 2 * (int)__popcll(eq[d] & pm) - (int)__popcll(ex[d] & pm);
        }
    }
    // the x-bond of x = wx-1 leaves the tile: shifted out by the mask
    const uint64_t SS = rowok ? (~(opn[0] << 1) & lbw) : 0ull;
    if (active && q == 0) {
        sm.SS[r] = SS;
        if (rowok && ((opn[0] >> (g.wx - 1)) & 1ull)) atomicOr(&sm.XF[r >> 5], 1u << (r & 31));
    }
    // crossing bits of the far y / z faces (y: bit x + TX*lz, z: x + TX*ly);
    // rows past the tile's extent write zeros
    {
        uint32_t* xb = R.xbits + (size_t)t * C::XW;
        if (active && edgeY && (xp & 31) == 0)
            xb[C::W0 + (C::TX * lz + xp) / 32] = rowok ? (uint32_t)(opn[1] >> xp) : 0u;
        if (C::D == 3 && active && edgeZ && (xp & 31) == 0)
            xb[C::W0 + C::W1 + (C::TX * ly + xp) / 32] = rowok ? (uint32_t)(opn[C::D - 1] >> xp) : 0u;
    }
    __syncthreads();

    // 3) unions between runs of neighbouring rows.  Within a stretch where
    //    neither row starts a new run both rows stay in the same two runs, so
    //    only the first open bond of each stretch is joined.  Each wave queues
    //    its unions and runs them 64 at a time, so the time goes with the
    //    wave's number of unions rather than with its busiest thread.
    {
        const int lane = tid & 63, wave = tid >> 6;
        uint32_t* ring = sm.ring[wave];
        uint32_t tail = 0, head = 0;
        // a queued union is (x, row, direction); its two run starts are found
        // when it is joined, where every lane of the wave has one
        auto join = [&](uint32_t e) {
            const int x = (int)(e & 63u), rr = (int)((e >> 6) & 63u);
            const int st = (e >> 12) ? C::TY : 1;
            lds_join(sm.par, rr * C::TX + start_at(sm.SS[rr], x), (rr + st) * C::TX + start_at(sm.SS[rr + st], x));
        };
#pragma unroll
        for (int dd = 1; dd < C::D; ++dd) {
            const bool inner = rowok && ((dd == 1) ? (ly < g.wy - 1) : (lz < g.wz - 1));
            uint32_t U16 = 0;                                    // this part's unions, bit j = site xp + j
            if (inner) {
                const uint64_t SSp = sm.SS[r + ((dd == 1) ? 1 : C::TY)];
                const uint64_t V = opn[dd];
                const uint64_t Mc = ~(SS | SSp);                 // neither row starts a run here
                const uint64_t A = V | Mc;
                const uint64_t carry = (A + V) ^ A ^ V;          // an open bond earlier in the stretch
                U16 = (uint32_t)((V & ~(Mc & carry)) >> xp) & 0xFFFFu;
            }
            const uint32_t tagbits = ((uint32_t)r << 6) | ((uint32_t)(dd - 1) << 12) | (uint32_t)xp;
            while (__ballot(U16 != 0u)) {
                const bool want = U16 != 0u;
                uint32_t e = 0;
                if (want) {
                    e = tagbits + (uint32_t)__builtin_ctz(U16);
                    U16 &= U16 - 1u;
                }
                const uint64_t bal = __ballot(want);
                if (want) ring[(tail + (uint32_t)lanes_below(bal)) & (kRing - 1)] = e;
                tail += (uint32_t)__popcll(bal);
                if (tail - head >= 64u) {
                    wave_lds_sync();
                    join(ring[(head + (uint32_t)lane) & (kRing - 1)]);
                    head += 64u;
                    wave_lds_sync();
                }
            }
        }
        wave_lds_sync();
        if ((uint32_t)lane < tail - head) join(ring[(head + (uint32_t)lane) & (kRing - 1)]);
    }
    __syncthreads();

    // 4) tile-local labels (the cluster's tile root) of the part and of its
    //    face sites, and border flags: a cluster is a border cluster when one
    //    of its runs touches a near face or has an open link leaving through a
    //    far face.  Every run start walks to its root once and stores it as
    //    its parent (the parents only change by such stores now, each of
    //    which writes an ancestor).  A thread keeps two walks in flight and
    //    starts its next run start as soon as one ends, so a wave waits about
    //    half as many LDS round trips as its busiest thread has steps.
    const int rowk = r * C::TX;
    const uint32_t ss16 = partok ? (uint32_t)(SS >> xp) & (uint32_t)low_bits(np) : 0u;   // run starts of the part
    {
        uint32_t pend = ss16;
        int sa = -1, na = 0, sb = -1, nb = 0;   // start and current node of the two walks (-1: idle)
        auto next = [&](int& st, int& nd) {
            if (pend) {
                st = rowk + xp + __builtin_ctz(pend);
                pend &= pend - 1u;
            } else {
                st = -1;
            }
            nd = st < 0 ? 0 : st;
        };
        next(sa, na);
        next(sb, nb);
        while (__ballot(sa >= 0 || sb >= 0)) {
            const int pa = lds_load(&sm.par[na]);   // idle walks read par[0], a root
            const int pb = lds_load(&sm.par[nb]);
            if (sa >= 0) {
                if (pa != na) {
                    na = pa;
                } else {
                    if (na != sa) lds_store(&sm.par[sa], na);
                    next(sa, na);
                }
            }
            if (sb >= 0) {
                if (pb != nb) {
                    nb = pb;
                } else {
                    if (nb != sb) lds_store(&sm.par[sb], nb);
                    next(sb, nb);
                }
            }
        }
    }
    wave_lds_sync();   // the run start before xp is a thread of the same row, so of this wave
    if (partok) {
        uint16_t* nearf = sm.fst;   // staged: they go out as ranks once the border roots are known
        uint16_t* farf = sm.fst + C::FT;
        const bool nearrow = ly == 0 || (C::D == 3 && lz == 0);
        uint64_t cross = 0;                                   // open links leaving through the far y / z faces
        if (edgeY) cross |= opn[1];
        if (edgeZ) cross |= opn[C::D - 1];
        const int last = 63 - __clzll((long long)SS);
        const bool xout = (opn[0] >> (g.wx - 1)) & 1ull;
        uint32_t rt[16];                                      // roots of the part's run starts
        {
            const uint4* pv = reinterpret_cast<const uint4*>(sm.par + rowk + xp);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint4 v = pv[k];
                rt[4 * k] = v.x;
                rt[4 * k + 1] = v.y;
                rt[4 * k + 2] = v.z;
                rt[4 * k + 3] = v.w;
            }
        }
        // border runs of the row as a mask of their run starts: every run of
        // a near row, the run at x = 0, the last run when its x-link leaves
        // the tile, and every run holding a link that leaves through a far y
        // / z face.  A run [s, e] holds a bit of `cross` when, in the
        // bit-reversed row (where the run is [63-e, 63-s] with its start on
        // top), a carry started at a reversed cross bit climbs to the top
        // through positions that are not a run's bottom (an end, reversed).
        uint64_t bs;
        if (nearrow) {
            bs = SS;
        } else {
            bs = 1ull | (xout ? (1ull << last) : 0ull);
            if (cross) {
                const uint64_t ends = ((SS >> 1) | (1ull << (g.wx - 1))) & lbw;
                const uint64_t y = __builtin_bitreverse64(cross & lbw);
                const uint64_t cont = ~__builtin_bitreverse64(ends);
                const uint64_t a = y | cont;
                const uint64_t carry = (a + y) ^ a ^ y;
                bs |= __builtin_bitreverse64(((carry & cont) | y) & __builtin_bitreverse64(SS));
            }
            bs &= SS;
        }
        for (uint32_t bm = (uint32_t)(bs >> xp) & ss16; bm; bm &= bm - 1u) {
            const uint32_t root = (uint32_t)lds_load(&sm.par[rowk + xp + __builtin_ctz(bm)]);
            atomicOr(&sm.FB[root >> 5], 1u << (root & 31u));
        }
        // the labels of the part: each site takes the root of its run
        uint32_t cur = (ss16 & 1u) ? rt[0] : (uint32_t)lds_load(&sm.par[rowk + start_at(SS, xp)]);
        uint32_t pk[8];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            cur = ((ss16 >> j) & 1u) ? rt[j] : cur;
            if (j & 1) pk[j >> 1] |= cur << 16;
            else pk[j >> 1] = cur;
        }
        const int yfi = C::F0 + C::TX * lz + xp;          // y faces: index x + TX*lz
        const int zfi = C::F0 + C::F1 + C::TX * ly + xp;  // z faces: index x + TX*ly
        if (wide) {
            const uint4 lo = make_uint4(pk[0], pk[1], pk[2], pk[3]);
            const uint4 hi = make_uint4(pk[4], pk[5], pk[6], pk[7]);
            uint4* dst = reinterpret_cast<uint4*>(R.lab16 + gi0 + (uint32_t)xp);
            dst[0] = lo;
            dst[1] = hi;
            if (ly == 0) { reinterpret_cast<uint4*>(nearf + yfi)[0] = lo; reinterpret_cast<uint4*>(nearf + yfi)[1] = hi; }
            if (edgeY) { reinterpret_cast<uint4*>(farf + yfi)[0] = lo; reinterpret_cast<uint4*>(farf + yfi)[1] = hi; }
            if (C::D == 3 && lz == 0) { reinterpret_cast<uint4*>(nearf + zfi)[0] = lo; reinterpret_cast<uint4*>(nearf + zfi)[1] = hi; }
            if (edgeZ) { reinterpret_cast<uint4*>(farf + zfi)[0] = lo; reinterpret_cast<uint4*>(farf + zfi)[1] = hi; }
        } else {
            for (int j = 0; j < np; ++j) {
                const uint16_t v = (uint16_t)(pk[j >> 1] >> (16 * (j & 1)));
                R.lab16[gi0 + (uint32_t)(xp + j)] = v;
                if (ly == 0) nearf[yfi + j] = v;
                if (edgeY) farf[yfi + j] = v;
                if (C::D == 3 && lz == 0) nearf[zfi + j] = v;
                if (edgeZ) farf[zfi + j] = v;
            }
        }
        if (q == 0) nearf[r] = (uint16_t)pk[0];                              // x faces: index ly + TY*lz
        if (xp <= g.wx - 1 && g.wx - 1 < xp + 16) {
            const int jl = g.wx - 1 - xp;
            farf[r] = (uint16_t)(pk[jl >> 1] >> (16 * (jl & 1)));
        }
    }
    __syncthreads();

    // 4a) ranks of the border roots (border roots before each bitmap word), and
    //     the face labels out as the ranks of their tile roots: the border
    //     merge then addresses the union-find slots directly.  With the
    //     topological rule the labels themselves go out.
    if (tid < 64) {
        constexpr int WPL = (C::FBW + 63) / 64;         // bitmap words per lane of wave 0
        int cnt[WPL];
        int tot = 0;
#pragma unroll
        for (int k = 0; k < WPL; ++k) {
            const int w = tid * WPL + k;
            cnt[k] = (w < C::FBW) ? __popc(sm.FB[w]) : 0;
            tot += cnt[k];
        }
        int inc = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(inc, off, 64);
            if (tid >= off) inc += v;
        }
        int ex = inc - tot;
#pragma unroll
        for (int k = 0; k < WPL; ++k) {
            const int w = tid * WPL + k;
            if (w < C::FBW) sm.pre[w] = ex;
            ex += cnt[k];
        }
    }
    __syncthreads();
    {
        const bool ranks = !(R.flags & FLAG_WIND);
        uint32_t* dst = reinterpret_cast<uint32_t*>(R.face + (size_t)t * (2 * C::FT));
        const uint32_t* src = reinterpret_cast<const uint32_t*>(sm.fst);
        for (int i = tid; i < C::FT; i += blockDim.x) {   // two face sites per thread and step
            uint32_t w = src[i];
            if (ranks) {
                uint32_t o = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t v = (w >> (16 * h)) & 0xFFFFu;
                    // entries of sites outside a ragged tile are never read: any value will do
                    const uint32_t rk = (v < (uint32_t)C::TS)
                                            ? (uint32_t)sm.pre[v >> 5] + __popc(sm.FB[v >> 5] & ((1u << (v & 31u)) - 1u))
                                            : 0xFFFFu;
                    o |= rk << (16 * h);
                }
                w = o;
            }
            dst[i] = w;
        }
    }

    // 4b) PCC: the columns and rows each border cluster occupies in the tile.
    //    A cluster that covers every coordinate of an axis meets the
    //    hyperplane x_a = 0 and so touches a near face of some tile: only
    //    border clusters can span.  Each run start of a border cluster ORs its
    //    run's columns and its row into the cluster's entry; a thread merges
    //    consecutive runs of one cluster before the LDS atomics.
    // (a batched launch runs this variant for every replica of a batch that
    // holds a PCC replica: only PCC replicas have coverage entries)
    if constexpr (PCC) if ((R.flags & (FLAG_PCC | FLAG_WIND)) == FLAG_PCC) {
        using CV = K1Cov<C, true>;
        __syncthreads();   // the staged face labels are read: their space takes the coverage entries
        for (int k = tid; k < CV::CAP; k += blockDim.x) sm.cov.a[k] = sm.cov.b[k] = 0ull;
        __syncthreads();
        if (partok) {
            const unsigned long long rowb = (C::D == 3) ? ((1ull << ly) | (1ull << (C::TY + lz))) : (1ull << ly);
            uint32_t m = ss16;
            int cr = -1;
            unsigned long long ca = 0, cb = 0;
            while (m) {
                const int j = __builtin_ctz(m);
                m &= m - 1u;
                const int x = xp + j;
                const uint32_t root = (uint32_t)lds_load(&sm.par[rowk + x]);   // the walk left the root here
                const uint32_t fw = sm.FB[root >> 5];
                if (!((fw >> (root & 31u)) & 1u)) continue;
                const int rank = sm.pre[root >> 5] + __popc(fw & ((1u << (root & 31u)) - 1u));
                if (rank >= CV::CAP) {
                    flag_error(R, ERR_TILE_LABEL);
                    continue;
                }
                const uint64_t later = SS & ~low_bits(x + 1);
                const int xe = later ? __builtin_ctzll(later) - 1 : g.wx - 1;   // last site of the run
                if (rank != cr) {
                    if (cr >= 0) {
                        atomicOr(&sm.cov.a[cr], ca);
                        atomicOr(&sm.cov.b[cr], cb);
                    }
                    cr = rank;
                    ca = cb = 0;
                }
                ca |= low_bits(xe + 1) & ~low_bits(x);
                cb |= rowb;
            }
            if (cr >= 0) {
                atomicOr(&sm.cov.a[cr], ca);
                atomicOr(&sm.cov.b[cr], cb);
            }
        }
        __syncthreads();
        const int nb = sm.pre[C::FBW - 1] + __popc(sm.FB[C::FBW - 1]);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(R.cov) + (size_t)t * (2 * CV::CAP);
        for (int k = tid; k < nb && k < CV::CAP; k += blockDim.x) {
            dst[2 * k] = sm.cov.a[k];
            dst[2 * k + 1] = sm.cov.b[k];
        }
    }

    // 5) the border bitmap (and for PCC its ranks) and the far x face's
    //    crossing bits; every border root starts its own tree in the border
    //    merge's union-find, at its slot
    const bool wind = (R.flags & FLAG_WIND) != 0;
    for (int w = tid; w < C::FBW; w += blockDim.x) {
        R.fbits[(size_t)t * C::FBW + w] = sm.FB[w];
        if (R.fpre) R.fpre[(size_t)t * C::FBW + w] = (uint16_t)sm.pre[w];
    }
    constexpr int CAP = 2 * C::FT;   // a border root has a site on a near face or a far-face link
    const uint32_t slot0 = (uint32_t)t * (uint32_t)CAP;
    for (int hw = tid; hw < 2 * C::FBW; hw += blockDim.x) {   // 16 bits per thread
        const uint32_t word = sm.FB[hw >> 1];
        uint32_t m = (word >> (16 * (hw & 1))) & 0xFFFFu;
        int rank = sm.pre[hw >> 1] + ((hw & 1) ? __popc(word & 0xFFFFu) : 0);
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1u;
            const uint32_t gi = local_to_global<C>((uint32_t)(hw * 16 + b), g.x0, g.y0, g.z0, (int)L);
            if (wind) {
                R.par64[gi] = (uint64_t)gi;   // own root, sheet offset 0
            } else if (rank < CAP) {
                R.dpar[slot0 + (uint32_t)rank] = pack_node(gi, slot0 + (uint32_t)rank);
            } else {
                flag_error(R, ERR_TILE_LABEL);
            }
            ++rank;
        }
    }
    if (tid < C::W0) R.xbits[(size_t)t * C::XW + tid] = sm.XF[tid];
    __syncthreads();
}

// --------------------------------------------------------------------------
// K2: border merge.  For each far-face site of a tile whose link across the
// face is open, the two tile-local roots it joins are united in the global
// union-find.  Face labels come from the compact face arrays.
// --------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ uint32_t tile_site_global(const SwRep& R, int ix, int iy, int iz, uint32_t lr)
{
    return local_to_global<C>(lr, ix * C::TX, iy * C::TY, iz * C::TZ, R.L);
}

// K2 works one tile per workgroup.  Many open links across a face join the
// same two tile-local clusters; every distinct (face, near label, far label)
// triple is entered in an LDS hash set and only its first link makes the
// global union.  The work goes in three steps: the crossing bits are staged
// in LDS; each thread issues the label loads of all its face sites at once
// and enters its open links in the set, the first link of each triple going
// to a compact list; the unions of the list are then spread over all
// threads, so that a thread waits for about one union instead of one per
// face site it owns.
constexpr uint32_t kK2Empty = 0xFFFFFFFFu;

template <class C>
struct K2Cfg {
    static constexpr int NT = (C::FT <= 128) ? 64 : kBlock;    // default threads per tile: one wave when the far faces are small (more tiles in flight)
    static constexpr int HBITS = (2 * C::FT <= 256) ? 8 : (2 * C::FT <= 512) ? 9 : (2 * C::FT <= 1024) ? 10
                               : (2 * C::FT <= 2048) ? 11 : 12;
    static constexpr int H = 1 << HBITS;   // hash slots: at least twice the face sites
    static_assert(H >= 2 * C::FT, "hash set too small");
};

template <class C>
struct K2Smem {
    uint32_t keys[K2Cfg<C>::H];
    uint32_t list[C::FT];      // keys of the unions to make (at most one per face site)
    int cnt;
};

// true for the first caller with this key (keys < 2^28; the set is never full)
template <class C>
__device__ __forceinline__ bool k2_first(K2Smem<C>& sm, uint32_t key)
{
    constexpr uint32_t mask = K2Cfg<C>::H - 1;
    uint32_t h = (key * 0x9E3779B1u) >> (32 - K2Cfg<C>::HBITS);
    while (true) {
        const uint32_t old = atomicCAS(&sm.keys[h], kK2Empty, key);
        if (old == kK2Empty) return true;
        if (old == key) return false;
        h = (h + 1u) & mask;
    }
}

// face set (0 x, 1 y, 2 z) of far-face index f, its index within the set
// and the first crossing-bit word of the set
template <class C>
__device__ __forceinline__ void k2_face(int f, int& d, int& fb, int& wbase)
{
    if (f < C::F0) {
        d = 0;
        fb = f;
        wbase = 0;
    } else if (f < C::F0 + C::F1) {
        d = 1;
        fb = f - C::F0;
        wbase = C::W0;
    } else {
        d = 2;
        fb = f - C::F0 - C::F1;
        wbase = C::W0 + C::W1;
    }
}

// The merge schedule: NT threads per tile (the launch's workgroup size, 64 or
// 256), each with KF far-face sites; the autotuner picks NT.
template <class C, int NT>
struct K2Width {
    static constexpr int KF = (C::FT + NT - 1) / NT;           // face sites per thread
    static constexpr int H = K2Cfg<C>::H;
};

template <class C, int NT>
__device__ void k2_tile(const SwRep& R, int t, K2Smem<C>& sm)
{
    using K = K2Width<C, NT>;
    const int tid = threadIdx.x, nt = NT;
    for (int i = tid; i < K::H; i += nt) sm.keys[i] = kK2Empty;
    if (tid == 0) sm.cnt = 0;
    const int ix = t % R.ntx, iy = (t / R.ntx) % R.nty, iz = t / (R.ntx * R.nty);
    const uint16_t* farf = R.face + (size_t)t * (2 * C::FT) + C::FT;
    const uint32_t* xbt = R.xbits + (size_t)t * C::XW;
    // 1) the labels at both ends of every open link of this thread's face
    //    sites: the crossing bits and both face arrays are read together (the
    //    labels of closed links are read too and dropped), so that one round
    //    trip to memory brings all three
    uint32_t la[K::KF], lb[K::KF];
    int dk[K::KF];
    bool open[K::KF];
#pragma unroll
    for (int k = 0; k < K::KF; ++k) {
        const int f = tid + k * nt;
        open[k] = false;
        dk[k] = 0;
        la[k] = lb[k] = 0u;
        if (f < C::FT) {
            int d, fb, wbase;
            k2_face<C>(f, d, fb, wbase);
            dk[k] = d;
            int jx = ix, jy = iy, jz = iz;
            if (d == 0) jx = (ix + 1 == R.ntx) ? 0 : ix + 1;
            else if (d == 1) jy = (iy + 1 == R.nty) ? 0 : iy + 1;
            else jz = (iz + 1 == R.ntz) ? 0 : iz + 1;
            const int tn = jx + R.ntx * (jy + R.nty * jz);
            const uint32_t xw = xbt[wbase + (fb >> 5)];
            la[k] = farf[f];
            lb[k] = R.face[(size_t)tn * (2 * C::FT) + f];
            open[k] = (xw >> (fb & 31)) & 1u;
        }
    }
    __syncthreads();   // the hash set is cleared
    // 2) the first link of each (face, near label, far label) triple; the
    //    labels are the ranks of the two tile roots among their tiles' border
    //    roots (with the topological rule, the tile-local labels)
    const bool wind = (R.flags & FLAG_WIND) != 0;
    const uint32_t lim = wind ? (uint32_t)C::TS : (uint32_t)(2 * C::FT);
#pragma unroll
    for (int k = 0; k < K::KF; ++k) {
        if (!open[k]) continue;
        if (la[k] >= lim || lb[k] >= lim) {
            flag_error(R, ERR_TILE_LABEL);
            continue;
        }
        const uint32_t key = la[k] | (lb[k] << 13) | ((uint32_t)dk[k] << 26);
        if (k2_first<C>(sm, key)) sm.list[atomicAdd(&sm.cnt, 1)] = key;
    }
    __syncthreads();
    // 3) the unions, spread over the workgroup
    const int n = sm.cnt;
    for (int i = tid; i < n; i += nt) {
        const uint32_t key = sm.list[i];
        const uint32_t la0 = key & 0x1FFFu, lb0 = (key >> 13) & 0x1FFFu;
        const int d = (int)(key >> 26);
        int jx = ix, jy = iy, jz = iz;
        if (d == 0) jx = (ix + 1 == R.ntx) ? 0 : ix + 1;
        else if (d == 1) jy = (iy + 1 == R.nty) ? 0 : iy + 1;
        else jz = (iz + 1 == R.ntz) ? 0 : iz + 1;
        const int tn = jx + R.ntx * (jy + R.nty * jz);
        if (!wind) {
            constexpr uint32_t CAP = 2 * C::FT;
            d_unite(R, (uint32_t)t * CAP + la0, ~0u, (uint32_t)tn * CAP + lb0, ~0u);
            continue;
        }
        const uint32_t ra = tile_site_global<C>(R, ix, iy, iz, la0);
        const uint32_t rb = tile_site_global<C>(R, jx, jy, jz, lb0);
        if (ra >= R.N || rb >= R.N) {
            flag_error(R, ERR_TILE_LABEL);
            continue;
        }
        {
            // the link leaves the box's last tile along d: it wraps
            const bool wraps = (d == 0) ? ix + 1 == R.ntx : (d == 1) ? iy + 1 == R.nty : iz + 1 == R.ntz;
            Sheet w{{0, 0, 0}};
            if (wraps) w.v[d] = 1;
            g_unite64(R, ra, rb, w);
        }
    }
    __syncthreads();
}

// atomicOr(addr, bits) for every lane with `pending`, combined over the wave:
// lanes with the same target word OR their bits into the wave's LDS word and
// one of them makes the global atomic.  All lanes of the wave must call it.
__device__ __forceinline__ void wave_or(uint32_t* addr, uint32_t bits, bool pending, uint32_t* wscr)
{
    const int lane = threadIdx.x & 63;
    while (true) {
        const uint64_t bal = __ballot(pending);
        if (!bal) break;
        const int first = __builtin_ctzll(bal);
        const uint64_t lead = __shfl((uint64_t)(uintptr_t)addr, first, 64);
        bool leader = false;
        if (pending && (uint64_t)(uintptr_t)addr == lead) {
            atomicOr(wscr, bits);
            pending = false;
            leader = lane == first;
        }
        wave_lds_sync();
        if (leader) {
            atomicOr(addr, *wscr);
            *wscr = 0;
        }
        wave_lds_sync();
    }
}

// --------------------------------------------------------------------------
// K3a: border roots and the tile's flip bitmap, one wave per tile.  The roots
// in the tile's border bitmap are compacted into a list; each lane takes one
// at a time, finds its cluster root (the smallest site index of the cluster:
// the label identity that the min-label rule of Sec. II.B converges to),
// keeps it as parent when labels are written, and records the cluster's flip
// bit.  Each lane also draws the flip bits of one tile row: an interior root
// is its own cluster's label, so its bit is the one drawn for its own site.
// The result is one bit per tile-local site, meaningful at the tile roots.
// --------------------------------------------------------------------------
template <class C>
struct K3aSmem {
    uint16_t list[2 * C::FT];    // the tile's border roots in bitmap order (each has a site on a face)
    uint32_t root[2 * C::FT];    // their cluster roots (PCC coverage marks)
    uint32_t BF[C::FBW];         // flip bits of the border roots
    uint32_t FBt[C::FBW];        // the border-root bitmap
    uint32_t wor;                // word for combining coverage marks over the wave
};

// PCC coverage marks (extension rule, Sec. III): every border root of the
// tile whose cluster is a candidate of axis a in this sweep (it meets the
// hyperplane x_a = 0; k_cand_tile gave it a slot) ORs the axis-a coordinates
// its tile cluster occupies (K1's coverage entry, shifted to the tile's
// origin) into the slot's bitmap.  Marks of one bitmap word are combined over
// the wave before the global atomic; every lane runs the same iterations.
// (The axis loop stays rolled, and the callers make one call after the tile's
// K3a with the dimension as data: unrolled, or inlined once per dimension in
// the batched kernel, its wave-combining loops triple the register count of
// every K3a.)
struct CovArgs {
    int32_t dim, ty;                 // dimension and tile extent in y (bits of y in the row word)
    uint32_t L, N, s;
    int32_t x0, y0, z0, wx, wy, wz;
    const uint64_t* cand;
    uint32_t* bmp;
    const unsigned long long* cov;   // the tile's coverage entries
    int32_t* err;
    int nl;                          // border roots of the tile
    const uint32_t* roots;           // their cluster roots (LDS)
    uint32_t* wscr;                  // LDS word for combining marks over the wave
};

static __device__ __forceinline__ void k3a_coverage(const CovArgs& A)
{
    const int lane = threadIdx.x & 63;
    const int nl = A.nl;
    const uint64_t tag = (uint64_t)(A.s + 1u) << 32;
    const uint32_t bw = (A.L + 31u) / 32u;
    const uint32_t nslots = (A.dim == 3) ? A.L * A.L : A.L;
    wave_lds_sync();
    for (int base = 0; base < nl; base += 64) {
        const int k = base + lane;
        const bool valid = k < nl;
        const uint32_t root = valid ? A.roots[k] : 0u;
        const unsigned long long ca = valid ? A.cov[2 * k] : 0ull, cb = valid ? A.cov[2 * k + 1] : 0ull;
#pragma unroll 1
        for (int a = 0; a < A.dim; ++a) {
            bool cand = false;
            uint32_t slot = 0;
            if (valid && root < A.N) {
                const uint64_t c = A.cand[(size_t)a * A.N + root];
                if ((c & 0xFFFFFFFF00000000ull) == tag) {
                    slot = ~(uint32_t)c;
                    if (slot < nslots) cand = true;
                    else if (A.err) atomicOr(A.err, 1 << ERR_SLOT);
                }
            }
            // this cluster's axis-a coordinates in the tile, from the tile's
            // origin on (masked to the tile's extent, so that no mark can
            // leave the bitmap)
            uint64_t bits;
            uint32_t c0;
            if (a == 0) {
                bits = ca & low_bits(A.wx);
                c0 = (uint32_t)A.x0;
            } else if (a == 1) {
                bits = cb & low_bits(A.wy);
                c0 = (uint32_t)A.y0;
            } else {
                bits = (cb >> A.ty) & low_bits(A.wz);
                c0 = (uint32_t)A.z0;
            }
            // tile origins are multiples of the extent (32 / 64 in x, 64 in 2D y,
            // 8 in 3D y and z), so the shifted bits stay within two words
            const uint64_t sb = bits << (c0 & 31u);
            uint32_t* row = A.bmp + ((size_t)a * nslots + slot) * bw + (c0 >> 5);
            const uint32_t lo = (uint32_t)sb, hi = (uint32_t)(sb >> 32);
            wave_or(row, lo, cand && lo != 0u, A.wscr);
            wave_or(row + 1, hi, cand && hi != 0u, A.wscr);
        }
    }
}

// Returns, for PCC replicas, the arguments of the coverage marks (cov.nl < 0:
// none to make); the caller runs k3a_coverage after it.
template <class C>
__device__ void k3a_tile(const SwRep& R, int t, uint32_t s, K3aSmem<C>& sm, CovArgs& cov)
{
    constexpr int CAP = 2 * C::FT;
    const int lane = threadIdx.x & 63;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
    const bool keep = R.lab32 != nullptr;
    const bool pcc = (R.flags & (FLAG_PCC | FLAG_WIND)) == FLAG_PCC;   // extension rule or open-box spanning
    static_assert(C::NR == 64, "one tile row per lane");
    // the border roots in bitmap order (rank order, the order of K1's
    // coverage entries): lane l takes words [l * WPL, (l + 1) * WPL)
    constexpr int WPL = (C::FBW + 63) / 64;
    uint32_t mw[WPL];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int w = lane * WPL + k;
        mw[k] = (w < C::FBW) ? R.fbits[(size_t)t * C::FBW + w] : 0u;
        if (w < C::FBW) {
            sm.FBt[w] = mw[k];
            sm.BF[w] = 0;
        }
        tot += __popc(mw[k]);
    }
    int inc = tot;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(inc, off, 64);
        if (lane >= off) inc += v;
    }
    const int nb = __shfl(inc, 63, 64);
    int pos = inc - tot;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        uint32_t m = mw[k];
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1u;
            if (pos < CAP) sm.list[pos] = (uint16_t)((lane * WPL + k) * 32 + b);
            ++pos;
        }
    }
    if (lane == 0) sm.wor = 0;
    wave_lds_sync();
    uint64_t rf = 0;   // flip bits of this lane's row
    {
        const int ly = lane % C::TY, lz = lane / C::TY;
        if (ly < g.wy && lz < g.wz)
            rf = row_flips((uint32_t)g.x0 + (uint32_t)R.L * ((uint32_t)(g.y0 + ly) + (uint32_t)R.L * (uint32_t)(g.z0 + lz)),
                           g.wx, s, k0, k1);
    }
    if (nb > CAP && lane == 0) flag_error(R, ERR_TILE_LABEL);   // more border roots than face sites
    const int nl = min(nb, CAP);
    // two list entries per lane and step (i and i + 64), their finds together
    for (int i = lane; i < nl; i += 128) {
        const bool two = i + 64 < nl;
        uint32_t lr[2], gi[2], root[2];
        lr[0] = sm.list[i];
        lr[1] = two ? sm.list[i + 64] : lr[0];
#pragma unroll
        for (int e = 0; e < 2; ++e) gi[e] = local_to_global<C>(lr[e], g.x0, g.y0, g.z0, R.L);
        if (gi[0] >= R.N || gi[1] >= R.N) {
            flag_error(R, ERR_TILE_LABEL);
            continue;
        }
        root[0] = gi[0];
        root[1] = gi[1];
        if (R.flags & FLAG_WIND) {
            ro_find2(R, root[0], root[1]);
        } else {
            const uint32_t slot0 = (uint32_t)t * (uint32_t)CAP;   // list entry i holds slot t * CAP + i
            d_ro_find2(R, slot0 + (uint32_t)i, root[0], slot0 + (uint32_t)(two ? i + 64 : i), root[1]);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (e == 1 && !two) break;
            if (keep) R.par[gi[e]] = (int32_t)root[e];
            if (flip_bit(root[e], s, k0, k1)) atomicOr(&sm.BF[lr[e] >> 5], 1u << (lr[e] & 31u));
            sm.root[i + 64 * e] = root[e];
        }
    }
    wave_lds_sync();
    constexpr int WPR = C::TX / 32;   // bitmap words per row
#pragma unroll
    for (int k = 0; k < WPR; ++k) {
        const int w = lane * WPR + k;
        const uint32_t fb = sm.FBt[w];
        R.bflip[(size_t)t * C::FBW + w] = (fb & sm.BF[w]) | (~fb & (uint32_t)(rf >> (32 * k)));
    }
    cov.nl = -1;
    if (pcc)
        cov = CovArgs{C::D, C::TY, (uint32_t)R.L, R.N, s, g.x0, g.y0, g.z0, g.wx, g.wy, g.wz, R.cand, R.bmp,
                      reinterpret_cast<const unsigned long long*>(R.cov) + (size_t)t * (2 * CAP), R.err, nl, sm.root,
                      &sm.wor};
}

// --------------------------------------------------------------------------
// K3b: cluster flip.  Every site takes the flip bit that K3a recorded for its
// tile root and gets its cluster's new spin.  Optionally writes the final
// labels.
// --------------------------------------------------------------------------
template <class C>
struct K3Smem {
    uint32_t FL[C::FBW];         // flip bit of every tile root (from K3a)
    uint32_t FBt[C::FBW];        // the tile's border-root bitmap (labels only)
    uint32_t wbits[2 * (kK3Block / 64)];   // per wave: bits and set bits of the packed word being written
};

// new spin byte of the site with tile-local index k and stored label v;
// writes the final label when asked for
template <class C>
__device__ __forceinline__ uint32_t k3_site(const SwRep& R, const K3Smem<C>& sm, const TileGeo& g, uint32_t v, int k,
                                            uint32_t gi, bool labels)
{
    const uint32_t lr = v;
    if (lr > (uint32_t)k) {                 // a tile root precedes its sites
        flag_error(R, ERR_TILE_LABEL);
        return 0xFFu;
    }
    const uint32_t bit = (sm.FL[lr >> 5] >> (lr & 31u)) & 1u;
    if (labels) {
        const bool border = (sm.FBt[lr >> 5] >> (lr & 31u)) & 1u;
        uint32_t root = local_to_global<C>(lr, g.x0, g.y0, g.z0, R.L);
        if (border) root = (uint32_t)R.par[root];   // set to the cluster root by K3a
        if (root >= R.N) {
            flag_error(R, ERR_PARENT);
            root = 0;
        }
        R.lab32[gi] = (int32_t)root;
    }
    return bit ? 0x01u : 0xFFu;
}

// K3b when no final labels are asked for and rows are
// whole groups of W = 4 or 8 sites (the plain sweep): labels in, spins out,
// one bitmap word per site, W sites per load and store; the label check (a
// tile root precedes its sites) is folded into one flag per thread
template <class C, int W>
__device__ void k3_lean_tile(const SwRep& R, int t, const TileGeo& g, K3Smem<C>& sm)
{
    static_assert(W == 4 || W == 8, "groups of 4 or 8 sites");
    using LabV = typename std::conditional<W == 8, uint4, uint2>::type;   // W 16-bit labels
    using SpinV = typename std::conditional<W == 8, uint2, uint32_t>::type; // W spin bytes
    const int tid = threadIdx.x;
    const uint32_t L = (uint32_t)R.L;
    constexpr int GR = C::TX / W;                        // groups of sites per row
    constexpr int GPT = C::TS / W / kK3Block;            // groups per thread (blockDim = kK3Block)
    static_assert(C::TS % (W * kK3Block) == 0, "whole groups per thread");
    static_assert((C::TS & (C::TS - 1)) == 0, "a label masked to TS - 1 stays inside the bitmap");
    const bool packed = (R.flags & FLAG_BITPACK) != 0;   // then W = 8: one byte of bits per group
    LabV lv[GPT];
    uint32_t gq[GPT];
    bool ok[GPT];
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int qd = tid + kK3Block * j;
        const int r = qd / GR, xq = (qd % GR) * W;
        const int ly = r % C::TY, lz = r / C::TY;
        ok[j] = ly < g.wy && lz < g.wz && xq < g.wx;
        gq[j] = (uint32_t)(g.x0 + xq) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
        if (ok[j]) lv[j] = *reinterpret_cast<const LabV*>(R.lab16 + gq[j]);
        else lv[j] = LabV{};
    }
    for (int w = tid; w < C::FBW; w += blockDim.x) sm.FL[w] = R.bflip[(size_t)t * C::FBW + w];
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        const int qd = tid + kK3Block * j;
        const uint32_t k = (uint32_t)((qd / GR) * C::TX + (qd % GR) * W);
        const uint32_t* lw = reinterpret_cast<const uint32_t*>(&lv[j]);   // two labels per word
        uint32_t out[W / 4];
        uint32_t pb = 0;                                  // the group's new spins as bits
#pragma unroll
        for (int h = 0; h < W / 4; ++h) {
            out[h] = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = 4 * h + i;
                const uint32_t lab = (n & 1) ? lw[n >> 1] >> 16 : lw[n >> 1] & 0xFFFFu;
                bad |= lab > k + (uint32_t)n;
                const uint32_t lr = lab & (uint32_t)(C::TS - 1);
                const uint32_t bit = (sm.FL[lr >> 5] >> (lr & 31u)) & 1u;
                out[h] |= (bit ? 0x01u : 0xFFu) << (8 * i);
                pb |= bit << n;
            }
        }
        if (ok[j]) {
            if (packed)   // W = 8 sites from a multiple of 8: one byte of the packed array, owned by this tile
                reinterpret_cast<uint8_t*>(R.spins)[gq[j] >> 3] = (uint8_t)pb;
            else
                *reinterpret_cast<SpinV*>(R.spins + gq[j]) = *reinterpret_cast<const SpinV*>(out);
        }
    }
    if (bad) flag_error(R, ERR_TILE_LABEL);
    __syncthreads();
}

// K3b when no final labels are asked for and rows are not whole quads of
// sites (int8 spins).  A tile row's stretch of the spin array then starts
// anywhere in a 4-byte word: each thread takes one aligned word of a row (a
// row spans at most TX/4 + 1 of them), loads the four labels under it with
// one aligned 8-byte load (labels of the neighbouring tile's sites are read
// and ignored), and stores the word whole when all four sites are the tile's,
// else only the bytes that are.  The label check is folded as in the lean path.
template <class C>
__device__ void k3_word_lean_tile(const SwRep& R, int t, const TileGeo& g, K3Smem<C>& sm)
{
    const int tid = threadIdx.x;
    const uint32_t L = (uint32_t)R.L;
    constexpr int WR = C::TX / 4 + 1;                     // aligned words a row can touch
    constexpr int NW = C::NR * WR;
    constexpr int WPT = (NW + kK3Block - 1) / kK3Block;   // words per thread (blockDim = kK3Block)
    static_assert((C::TS & (C::TS - 1)) == 0, "a label masked to TS - 1 stays inside the bitmap");
    uint2 lv[WPT];
    uint32_t wa[WPT];   // the word's first site
    uint32_t lo[WPT];   // tile-local index of that site (may be below the row's first: then it wraps)
    uint32_t inm[WPT];  // bit i: site wa + i belongs to the tile's row
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int q = tid + kK3Block * j;
        const int r = q / WR, wi = q % WR;
        const int ly = r % C::TY, lz = r / C::TY;
        inm[j] = 0u;
        lv[j] = make_uint2(0u, 0u);
        wa[j] = 0u;
        lo[j] = 0u;
        if (q < NW && ly < g.wy && lz < g.wz) {
            const uint32_t a0 = (uint32_t)g.x0 + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
            const uint32_t a1 = a0 + (uint32_t)g.wx;
            const uint32_t w = (a0 & ~3u) + 4u * (uint32_t)wi;
            if (w < a1) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (w + (uint32_t)i >= a0 && w + (uint32_t)i < a1) inm[j] |= 1u << i;
                wa[j] = w;
                lo[j] = (uint32_t)(r * C::TX) + (w - a0);   // modulo 2^32 when w < a0
                lv[j] = *reinterpret_cast<const uint2*>(R.lab16 + w);   // the label array holds N rounded up to 4
            }
        }
    }
    for (int w = tid; w < C::FBW; w += blockDim.x) sm.FL[w] = R.bflip[(size_t)t * C::FBW + w];
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        if (!inm[j]) continue;
        uint32_t out = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t lab = (i & 1) ? ((i >> 1) ? lv[j].y : lv[j].x) >> 16 : ((i >> 1) ? lv[j].y : lv[j].x) & 0xFFFFu;
            const bool mine = (inm[j] >> i) & 1u;
            bad |= mine && lab > lo[j] + (uint32_t)i;
            const uint32_t lr = lab & (uint32_t)(C::TS - 1);
            const uint32_t bit = (sm.FL[lr >> 5] >> (lr & 31u)) & 1u;
            out |= (bit ? 0x01u : 0xFFu) << (8 * i);
        }
        if (inm[j] == 0xFu) {
            *reinterpret_cast<uint32_t*>(R.spins + wa[j]) = out;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if ((inm[j] >> i) & 1u) R.spins[wa[j] + (uint32_t)i] = (int8_t)(out >> (8 * i));
        }
    }
    if (bad) flag_error(R, ERR_TILE_LABEL);
    __syncthreads();
}

// The new spins of a bit-packed lattice, one site per thread: the bits of one
// 32-bit word are combined over the wave, and the word is updated with an
// atomic AND of its cleared bits then an OR of its set bits, so that tiles
// whose sites share a word (rows that are not whole words) never overwrite
// each other's bits.  All lanes of the wave call it.
__device__ __forceinline__ void wave_set_bits(uint32_t* words, uint32_t site, uint32_t up, bool pending, uint32_t* wscr)
{
    const int lane = threadIdx.x & 63;
    while (true) {
        const uint64_t bal = __ballot(pending);
        if (!bal) break;
        const int first = __builtin_ctzll(bal);
        const uint32_t lead = __shfl(site >> 5, first, 64);
        bool leader = false;
        if (pending && (site >> 5) == lead) {
            atomicOr(&wscr[0], 1u << (site & 31u));
            if (up) atomicOr(&wscr[1], 1u << (site & 31u));
            pending = false;
            leader = lane == first;
        }
        wave_lds_sync();
        if (leader) {
            const uint32_t m = wscr[0], v = wscr[1];
            if (m & ~v) atomicAnd(&words[lead], ~(m & ~v));
            if (v) atomicOr(&words[lead], v);
            wscr[0] = wscr[1] = 0;
        }
        wave_lds_sync();
    }
}

template <class C>
__device__ void k3_packed_tile(const SwRep& R, int t, const TileGeo& g, K3Smem<C>& sm, bool labels)
{
    const int tid = threadIdx.x;
    const uint32_t L = (uint32_t)R.L;
    if (tid < 2 * (kK3Block / 64)) sm.wbits[tid] = 0;
    for (int w = tid; w < C::FBW; w += blockDim.x) {
        sm.FL[w] = R.bflip[(size_t)t * C::FBW + w];
        if (labels) sm.FBt[w] = R.fbits[(size_t)t * C::FBW + w];
    }
    __syncthreads();
    uint32_t* words = reinterpret_cast<uint32_t*>(R.spins);
    for (int k0 = 0; k0 < C::TS; k0 += kK3Block) {     // every lane of a wave runs the same iterations
        const int k = k0 + tid;
        const int xk = k % C::TX, r = k / C::TX;
        const int ly = r % C::TY, lz = r / C::TY;
        const bool valid = ly < g.wy && lz < g.wz && xk < g.wx;
        const uint32_t gi = (uint32_t)(g.x0 + xk) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
        uint32_t up = 0;
        if (valid) up = k3_site<C>(R, sm, g, R.lab16[gi], k, gi, labels) == 0x01u;
        wave_set_bits(words, gi, up, valid, &sm.wbits[2 * (tid >> 6)]);
    }
    __syncthreads();
}

// Inlined into every caller: left to itself the compiler keeps one
// out-of-line copy for the batched and persistent kernels, where the replica
// descriptor then arrives as a per-lane pointer and every field is a vector
// load (the batched flip ran at about 60% of the plain one's rate per site).
template <class C>
__device__ __forceinline__ void k3_tile(const SwRep& R, int t, uint32_t s, K3Smem<C>& sm)
{
    (void)s;
    const int tid = threadIdx.x;
    const TileGeo g = tile_geo<C>(R, t);
    const uint32_t L = (uint32_t)R.L;
    const bool labels = R.lab32 != nullptr;
    constexpr int QR = C::TX / 4;                       // quads of sites per row
    constexpr int QPT = C::TS / 4 / kK3Block;           // quads per thread (blockDim = kK3Block)
    const bool packed = (R.flags & FLAG_BITPACK) != 0;
    const bool quads = (L & 3u) == 0;                   // then every row and the tile width are multiples of 4
    if (!labels && quads && (!packed || (L & 7u) == 0)) {
        if ((L & 7u) == 0) k3_lean_tile<C, 8>(R, t, g, sm);
        else k3_lean_tile<C, 4>(R, t, g, sm);
        return;
    }
    if (!labels && !packed) {   // rows that are not whole quads of sites
        k3_word_lean_tile<C>(R, t, g, sm);
        return;
    }
    if (packed) {                                        // labels, or rows that are not whole bytes of bits
        k3_packed_tile<C>(R, t, g, sm, labels);
        return;
    }

    // 0) the tile's labels, four sites per thread and load, issued first so
    //    that they arrive while the flip bitmap is staged
    uint2 lv[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int qd = tid + kK3Block * j;
        const int r = qd / QR, xq = (qd % QR) * 4;
        const int ly = r % C::TY, lz = r / C::TY;
        lv[j] = make_uint2(0u, 0u);
        if (quads && ly < g.wy && lz < g.wz && xq < g.wx)
            lv[j] = *reinterpret_cast<const uint2*>(R.lab16 + (uint32_t)(g.x0 + xq) +
                                                    L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz)));
    }

    // 1) the tile's flip bitmap (from K3a), and its border bitmap when the
    //    cluster roots are needed
    for (int w = tid; w < C::FBW; w += blockDim.x) {
        sm.FL[w] = R.bflip[(size_t)t * C::FBW + w];
        if (labels) sm.FBt[w] = R.fbits[(size_t)t * C::FBW + w];
    }
    __syncthreads();

    // 2) new spins (and final labels)
    if (quads) {
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int qd = tid + kK3Block * j;
            const int r = qd / QR, xq = (qd % QR) * 4;
            const int ly = r % C::TY, lz = r / C::TY;
            const bool valid = ly < g.wy && lz < g.wz && xq < g.wx;
            if (!valid) continue;
            const uint32_t gi = (uint32_t)(g.x0 + xq) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
            const uint2 v = lv[j];
            const int k = r * C::TX + xq;
            uint32_t out = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t vi = (i == 0) ? (v.x & 0xFFFFu) : (i == 1) ? (v.x >> 16) : (i == 2) ? (v.y & 0xFFFFu) : (v.y >> 16);
                out |= k3_site<C>(R, sm, g, vi, k + i, gi + (uint32_t)i, labels) << (8 * i);
            }
            *reinterpret_cast<uint32_t*>(R.spins + gi) = out;
        }
    } else {
        // rows that are not whole quads of sites: each thread takes four
        // consecutive sites of a row (the index arithmetic once per group),
        // with per-site loads and stores
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int qd = tid + kK3Block * j;
            const int r = qd / QR, xq = (qd % QR) * 4;
            const int ly = r % C::TY, lz = r / C::TY;
            if (!(ly < g.wy && lz < g.wz && xq < g.wx)) continue;
            const uint32_t gi = (uint32_t)(g.x0 + xq) + L * ((uint32_t)(g.y0 + ly) + L * (uint32_t)(g.z0 + lz));
            const int k = r * C::TX + xq;
            const int nq = min(4, g.wx - xq);
            uint16_t lab[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) lab[i] = (i < nq) ? R.lab16[gi + (uint32_t)i] : 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < nq) R.spins[gi + (uint32_t)i] = (int8_t)k3_site<C>(R, sm, g, lab[i], k + i, gi + (uint32_t)i, labels);
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
            const uint32_t fw = R.fbits[(size_t)t * C::FBW + (v >> 5)];
            if ((fw >> (v & 31u)) & 1u) {   // a border root: its cluster's root through its slot
                const uint32_t rank = (uint32_t)R.fpre[(size_t)t * C::FBW + (v >> 5)] + __popc(fw & ((1u << (v & 31u)) - 1u));
                if (rank >= (uint32_t)(2 * C::FT)) {
                    flag_error(R, ERR_TILE_LABEL);
                    continue;
                }
                r = d_ro_find(R, (uint32_t)t * (uint32_t)(2 * C::FT) + rank, r);
            }
            // in-plane position
            uint32_t slot;
            if (C::D == 2) slot = (a == 0) ? (uint32_t)y : (uint32_t)x;
            else slot = (a == 0) ? (uint32_t)y + L * (uint32_t)z : (a == 1) ? (uint32_t)x + L * (uint32_t)z : (uint32_t)x + L * (uint32_t)y;
            atomicMax((unsigned long long*)&R.cand[(size_t)a * R.N + r], (unsigned long long)(tag | (uint64_t)(~slot)));
        }
    }
}

}  // namespace sw
