/*
 * sw_oracle.c -- plain, sequential CPU oracle for one Swendsen-Wang sweep of
 * the Ising model H = -J sum_<ij> s_i s_j (Lin & Zheng, Sec. I, steps 1-4) and
 * for the probability-changing-cluster feedback (Sec. III) with its
 * percolation tests: the extension rule and the topological (winding) rule on
 * periodic boxes, and the spanning test of open boxes.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header or
 * table with the GPU library: the Philox generator below is written here from
 * its published definition (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), independently of the library's copy.
 *
 * Everything is deliberately unoptimised: one Philox call per link, one byte
 * per bond, breadth-first search for the clusters.
 *
 * Boundary conditions: periodic in every axis, or open (Sec. III discusses
 * both): with open boundaries the links that would wrap around the box do not
 * exist; every other link keeps its index and so its random draw.
 *
 * Conventions (the paper is silent on them; the readings are listed in the
 * design notes):
 *   - N = L^dim sites, site index i = x + L*y (+ L*L*z), x fastest.
 *   - link (i,d) joins i and i + e_d (periodic in every axis), link index
 *     l = d*N + i.
 *   - spins are int8 +1 / -1.
 *   - random stream "SWRNG-1": Philox4x32-10 with key (seed lo, seed hi) and
 *     counter (c0, 0, sweep, tag), tags INIT=0, BOND=1, REFINE=2, FLIP=3.
 *   - canonical cluster label = minimum site index in the cluster.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_TAG_INIT 0u
#define ORC_TAG_BOND 1u
#define ORC_TAG_REFINE 2u
#define ORC_TAG_FLIP 3u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, Sec. 3-4): ten rounds of the 4-word S-box with the  */
/* two published multipliers; the key is bumped by the two Weyl constants    */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One output word of the stream: word w of Philox((c0, 0, sweep, tag), seed). */
static uint32_t orc_word(uint64_t seed, uint32_t c0, uint32_t sweep, uint32_t tag, int w)
{
    uint32_t ctr[4] = {c0, 0u, sweep, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[w];
}

/* ------------------------------------------------------------------------ */
/* Bond probability (Sec. I step 1): P = 1 - exp(-2J/T), turned into an      */
/* integer threshold thr = min(2^32, floor(P * 2^32)); a link is drawn open   */
/* when a uniform 32-bit integer u satisfies u < thr.                         */
/* ------------------------------------------------------------------------ */
uint64_t orc_threshold_from_p(double p)
{
    if (!(p > 0.0)) return 0;           /* also maps NaN to 0 */
    if (p >= 1.0) return 4294967296ull;
    double t = floor(ldexp(p, 32));
    return (uint64_t)t;
}

double orc_bond_probability(double J, double T)
{
    /* 1 - exp(-2J/T), evaluated without cancellation */
    return -expm1(-2.0 * J / T);
}

uint64_t orc_threshold(double J, double T)
{
    return orc_threshold_from_p(orc_bond_probability(J, T));
}

/* ------------------------------------------------------------------------ */
/* The three draws of the stream.                                             */
/* ------------------------------------------------------------------------ */

/* initial spin of site i: bit (i mod 32) of word ((i>>5) mod 4) of block i>>7 */
int orc_init_spin(uint64_t seed, uint32_t i)
{
    uint32_t w = orc_word(seed, i >> 7, 0u, ORC_TAG_INIT, (int)((i >> 5) & 3u));
    return ((w >> (i & 31u)) & 1u) ? +1 : -1;
}

/*
 * Bond decision for link l between two sites whose spins are equal or not.
 * The uniform 32-bit u is split as u = a*2^24 + b: a is byte (l mod 16) of
 * the BOND block l>>4, b the low 24 bits of word (l mod 4) of the REFINE
 * block l>>2.  u < thr is decided as written, by comparing a with thr>>24
 * first and b with thr mod 2^24 only when the high parts tie.
 */
int orc_bond_open(uint64_t seed, uint32_t sweep, uint64_t thr, uint32_t l, int equal)
{
    if (!equal) return 0;                        /* only equal neighbours bond */
    uint32_t k = l & 15u;
    uint32_t word = orc_word(seed, l >> 4, sweep, ORC_TAG_BOND, (int)(k >> 2));
    uint32_t a = (word >> (8u * (k & 3u))) & 0xFFu;
    uint64_t t_hi = thr >> 24;                   /* in [0, 256] */
    uint64_t t_lo = thr & 0xFFFFFFull;
    if ((uint64_t)a < t_hi) return 1;
    if ((uint64_t)a > t_hi) return 0;
    uint32_t b = orc_word(seed, l >> 2, sweep, ORC_TAG_REFINE, (int)(l & 3u)) & 0xFFFFFFu;
    return (uint64_t)b < t_lo;
}

/* new spin of every site of the cluster whose canonical label is r */
int orc_flip_spin(uint64_t seed, uint32_t sweep, uint32_t r)
{
    uint32_t w = orc_word(seed, r >> 7, sweep, ORC_TAG_FLIP, (int)((r >> 5) & 3u));
    return ((w >> (r & 31u)) & 1u) ? +1 : -1;
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry.                                                          */
/* ------------------------------------------------------------------------ */
static int64_t orc_nsites(int dim, int L)
{
    int64_t n = 1;
    for (int d = 0; d < dim; ++d) n *= L;
    return n;
}

/* i + e_d with periodic wrap */
static int64_t orc_forward(int dim, int L, int64_t i, int d)
{
    (void)dim;
    int64_t stride = 1;
    for (int k = 0; k < d; ++k) stride *= L;
    int64_t coord = (i / stride) % L;
    return (coord == L - 1) ? i - (int64_t)(L - 1) * stride : i + stride;
}

/* i - e_d with periodic wrap */
static int64_t orc_backward(int dim, int L, int64_t i, int d)
{
    (void)dim;
    int64_t stride = 1;
    for (int k = 0; k < d; ++k) stride *= L;
    int64_t coord = (i / stride) % L;
    return (coord == 0) ? i + (int64_t)(L - 1) * stride : i - stride;
}

int orc_validate(int dim, int L)
{
    if (dim != 2 && dim != 3) return -1;
    if (L < 3) return -1;
    int64_t n = orc_nsites(dim, L);
    if (n >= 2147483648ll) return -1;
    if ((int64_t)dim * n >= 4294967296ll) return -1;
    return 0;
}

void orc_init_spins(int dim, int L, uint64_t seed, int8_t *spins)
{
    int64_t n = orc_nsites(dim, L);
    for (int64_t i = 0; i < n; ++i) spins[i] = (int8_t)orc_init_spin(seed, (uint32_t)i);
}

/* ------------------------------------------------------------------------ */
/* Step 1: bonds.  open[d*N + i] = 1 when link (i,d) is a bond.               */
/* ------------------------------------------------------------------------ */
void orc_bonds(int dim, int L, uint64_t seed, uint32_t sweep, uint64_t thr,
               const int8_t *spins, uint8_t *open)
{
    int64_t n = orc_nsites(dim, L);
    for (int d = 0; d < dim; ++d) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = orc_forward(dim, L, i, d);
            int64_t l = (int64_t)d * n + i;
            open[l] = (uint8_t)orc_bond_open(seed, sweep, thr, (uint32_t)l, spins[i] == spins[j]);
        }
    }
}

/* The same with open boundaries: a link that would wrap around the box (from
 * coordinate L-1 along its axis) does not exist and is never a bond. */
void orc_bonds_open(int dim, int L, uint64_t seed, uint32_t sweep, uint64_t thr,
                    const int8_t *spins, uint8_t *open)
{
    int64_t n = orc_nsites(dim, L);
    int64_t stride = 1;
    for (int d = 0; d < dim; ++d) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t l = (int64_t)d * n + i;
            if ((i / stride) % L == L - 1) {
                open[l] = 0;
                continue;
            }
            int64_t j = i + stride;
            open[l] = (uint8_t)orc_bond_open(seed, sweep, thr, (uint32_t)l, spins[i] == spins[j]);
        }
        stride *= L;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 2: clusters.  Visiting sites in increasing index order and flooding  */
/* each unvisited one breadth-first labels every cluster with the smallest  */
/* index it contains (all smaller indices were labelled earlier).            */
/* Returns the number of clusters, or -1 on allocation failure.              */
/* ------------------------------------------------------------------------ */
int64_t orc_label_bfs(int dim, int L, const uint8_t *open, int32_t *labels)
{
    int64_t n = orc_nsites(dim, L);
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -1;
    for (int64_t i = 0; i < n; ++i) labels[i] = -1;
    int64_t nclusters = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (labels[i] >= 0) continue;
        ++nclusters;
        int64_t head = 0, tail = 0;
        labels[i] = (int32_t)i;
        queue[tail++] = (int32_t)i;
        while (head < tail) {
            int64_t u = queue[head++];
            for (int d = 0; d < dim; ++d) {
                int64_t f = orc_forward(dim, L, u, d);
                if (open[(int64_t)d * n + u] && labels[f] < 0) {
                    labels[f] = (int32_t)i;
                    queue[tail++] = (int32_t)f;
                }
                int64_t b = orc_backward(dim, L, u, d);
                if (open[(int64_t)d * n + b] && labels[b] < 0) {
                    labels[b] = (int32_t)i;
                    queue[tail++] = (int32_t)b;
                }
            }
        }
    }
    free(queue);
    return nclusters;
}

/* ------------------------------------------------------------------------ */
/* Step 3: every site takes the fresh spin drawn for its cluster's label.    */
/* ------------------------------------------------------------------------ */
void orc_flip(int dim, int L, uint64_t seed, uint32_t sweep, const int32_t *labels, int8_t *spins)
{
    int64_t n = orc_nsites(dim, L);
    for (int64_t i = 0; i < n; ++i)
        spins[i] = (int8_t)orc_flip_spin(seed, sweep, (uint32_t)labels[i]);
}

/* ------------------------------------------------------------------------ */
/* Observables of H = -J sum s_i s_j: E_int = sum over links of s_i s_j (so  */
/* H = -J E_int) and M = sum of s_i.                                          */
/* ------------------------------------------------------------------------ */
void orc_measure(int dim, int L, const int8_t *spins, int64_t *e_int, int64_t *m)
{
    int64_t n = orc_nsites(dim, L);
    int64_t e = 0, mm = 0;
    for (int64_t i = 0; i < n; ++i) {
        mm += spins[i];
        for (int d = 0; d < dim; ++d) e += (int64_t)spins[i] * spins[orc_forward(dim, L, i, d)];
    }
    *e_int = e;
    *m = mm;
}

/* With open boundaries E_int sums over the existing links only. */
void orc_measure_open(int dim, int L, const int8_t *spins, int64_t *e_int, int64_t *m)
{
    int64_t n = orc_nsites(dim, L);
    int64_t e = 0, mm = 0;
    for (int64_t i = 0; i < n; ++i) {
        mm += spins[i];
        int64_t stride = 1;
        for (int d = 0; d < dim; ++d) {
            if ((i / stride) % L != L - 1) e += (int64_t)spins[i] * spins[i + stride];
            stride *= L;
        }
    }
    *e_int = e;
    *m = mm;
}

/* ------------------------------------------------------------------------ */
/* One full sweep (Sec. I steps 1-3).  spins is updated in place; labels     */
/* (N entries) receives the canonical labels of this sweep's clusters.       */
/* Returns 0, or -1 on allocation failure.                                    */
/* ------------------------------------------------------------------------ */
int orc_sweep(int dim, int L, uint64_t seed, uint32_t sweep, uint64_t thr,
              int8_t *spins, int32_t *labels)
{
    int64_t n = orc_nsites(dim, L);
    uint8_t *open = (uint8_t *)malloc((size_t)(dim * n));
    if (!open) return -1;
    orc_bonds(dim, L, seed, sweep, thr, spins, open);
    int64_t nc = orc_label_bfs(dim, L, open, labels);
    free(open);
    if (nc < 0) return -1;
    orc_flip(dim, L, seed, sweep, labels, spins);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Extension rule with periodic boundaries (Sec. III): the configuration     */
/* percolates when one cluster's projection onto some axis covers all L      */
/* coordinates.  Clusters are gathered by label (counting sort), and the     */
/* projection of every cluster with at least L sites is tested axis by axis. */
/* Returns 1 / 0, or -1 on allocation failure.                                */
/* ------------------------------------------------------------------------ */
int orc_percolates(int dim, int L, const int32_t *labels)
{
    int64_t n = orc_nsites(dim, L);
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *members = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint8_t *covered = (uint8_t *)malloc((size_t)L);
    if (!start || !fill || !members || !covered) {
        free(start); free(fill); free(members); free(covered);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) start[labels[i] + 1]++;
    for (int64_t r = 0; r < n; ++r) start[r + 1] += start[r];
    for (int64_t r = 0; r < n; ++r) fill[r] = start[r];
    for (int64_t i = 0; i < n; ++i) members[fill[labels[i]]++] = i;

    int result = 0;
    for (int64_t r = 0; r < n && !result; ++r) {
        int64_t size = start[r + 1] - start[r];
        if (size < L) continue;                 /* cannot cover L coordinates */
        int64_t stride = 1;
        for (int axis = 0; axis < dim && !result; ++axis) {
            memset(covered, 0, (size_t)L);
            for (int64_t k = start[r]; k < start[r + 1]; ++k)
                covered[(members[k] / stride) % L] = 1;
            int all = 1;
            for (int c = 0; c < L; ++c) all &= covered[c];
            if (all) result = 1;
            stride *= L;
        }
    }
    free(start); free(fill); free(members); free(covered);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Spanning with open boundaries (Sec. III): the configuration percolates    */
/* when one cluster occupies both opposite boundaries of some axis, the      */
/* sites with coordinate 0 and the sites with coordinate L-1.                */
/* Returns 1 / 0, or -1 on allocation failure.                                */
/* ------------------------------------------------------------------------ */
int orc_spans_open(int dim, int L, const int32_t *labels)
{
    int64_t n = orc_nsites(dim, L);
    uint8_t *low = (uint8_t *)malloc((size_t)n);     /* label touches coordinate 0 of the axis */
    if (!low) return -1;
    int result = 0;
    int64_t stride = 1;
    for (int axis = 0; axis < dim && !result; ++axis) {
        memset(low, 0, (size_t)n);
        for (int64_t i = 0; i < n; ++i)
            if ((i / stride) % L == 0) low[labels[i]] = 1;
        for (int64_t i = 0; i < n && !result; ++i)
            if ((i / stride) % L == L - 1 && low[labels[i]]) result = 1;
        stride *= L;
    }
    free(low);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Topological rule (Sec. III): the configuration percolates when one        */
/* cluster winds around the periodic box along some axis.  Each cluster is   */
/* searched breadth-first from its smallest site, giving every site reached  */
/* an unwrapped position (a step along a link moves one unit along its axis, */
/* whether or not the link wraps around the box).  A link that reaches a     */
/* site already placed at a different unwrapped position closes a loop that  */
/* goes around the box: its positions differ by a nonzero multiple of L.     */
/* Returns 1 / 0, or -1 on allocation failure.                                */
/* ------------------------------------------------------------------------ */
int orc_winds(int dim, int L, const uint8_t *open)
{
    int64_t n = orc_nsites(dim, L);
    int64_t *pos = (int64_t *)malloc((size_t)n * 3 * sizeof(int64_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!pos || !seen || !queue) {
        free(pos); free(seen); free(queue);
        return -1;
    }
    int result = 0;
    for (int64_t start = 0; start < n && !result; ++start) {
        if (seen[start]) continue;
        int64_t head = 0, tail = 0;
        seen[start] = 1;
        for (int d = 0; d < 3; ++d) pos[3 * start + d] = 0;
        queue[tail++] = start;
        while (head < tail && !result) {
            int64_t u = queue[head++];
            for (int d = 0; d < dim && !result; ++d) {
                for (int dir = 0; dir < 2 && !result; ++dir) {
                    int64_t v = dir ? orc_forward(dim, L, u, d) : orc_backward(dim, L, u, d);
                    int64_t link = dir ? (int64_t)d * n + u : (int64_t)d * n + v;
                    if (!open[link]) continue;
                    int64_t want[3] = {pos[3 * u], pos[3 * u + 1], pos[3 * u + 2]};
                    want[d] += dir ? 1 : -1;
                    if (!seen[v]) {
                        seen[v] = 1;
                        for (int k = 0; k < 3; ++k) pos[3 * v + k] = want[k];
                        queue[tail++] = v;
                    } else if (pos[3 * v] != want[0] || pos[3 * v + 1] != want[1] || pos[3 * v + 2] != want[2]) {
                        result = 1;
                    }
                }
            }
        }
    }
    free(pos); free(seen); free(queue);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Feedback on the bond probability after sweep `sweep` (PCC, Sec. I and     */
/* Sec. III): p -= dp when percolating, p += dp otherwise, with              */
/* dp = dp0 * 2^-(sweep / halve_every), clamped to [0, 1]; the threshold of  */
/* the next sweep is recomputed from p.                                       */
/* ------------------------------------------------------------------------ */
void orc_pcc_update(double *p, uint64_t *thr, int percolating, uint32_t sweep,
                    double dp0, uint32_t halve_every)
{
    double dp = ldexp(dp0, -(int)(sweep / halve_every));
    double q = percolating ? (*p - dp) : (*p + dp);
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    *p = q;
    *thr = orc_threshold_from_p(q);
}

/* ------------------------------------------------------------------------ */
/* A run of `nsweeps` sweeps starting at sweep index s0.                      */
/*   series   (2*nsweeps or NULL): (E_int, M) after every sweep               */
/*   labels   (N or NULL): labels of the last sweep                           */
/*   perc     (nsweeps or NULL): percolation flag of every sweep (pcc only)   */
/*   p_trace  (nsweeps or NULL): p after every sweep's update (pcc only)      */
/* With pcc != 0 the threshold follows the feedback rule, starting from      */
/* *thr / *p; otherwise *thr is used unchanged.  Returns 0 or -1.             */
/* ------------------------------------------------------------------------ */
/* mode bits of orc_run_bc */
#define ORC_PCC 1      /* PCC feedback                                          */
#define ORC_OPEN 2     /* open boundaries (spanning: both opposite boundaries)  */
#define ORC_WIND 4     /* topological rule (periodic boundaries only)           */

/* As orc_run, with the boundary conditions and the percolation rule chosen by
 * `mode`: periodic boundaries take the extension rule, or with ORC_WIND the
 * topological rule; open boundaries take the spanning test of the open box. */
int orc_run_bc(int dim, int L, uint64_t seed, uint32_t s0, int32_t nsweeps,
               uint64_t *thr, double *p, int mode, double dp0, uint32_t halve_every,
               int8_t *spins, int64_t *series, int32_t *labels, int32_t *perc, double *p_trace)
{
    if (orc_validate(dim, L) != 0 || nsweeps < 0) return -1;
    if ((mode & ORC_PCC) && halve_every == 0) return -1;
    if ((mode & ORC_OPEN) && (mode & ORC_WIND)) return -1;
    int64_t n = orc_nsites(dim, L);
    int32_t *lab = labels ? labels : (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *open = (uint8_t *)malloc((size_t)(dim * n));
    if (!lab || !open) {
        if (!labels) free(lab);
        free(open);
        return -1;
    }
    int rc = 0;
    for (int32_t k = 0; k < nsweeps; ++k) {
        uint32_t sweep = s0 + (uint32_t)k;
        if (mode & ORC_OPEN) orc_bonds_open(dim, L, seed, sweep, *thr, spins, open);
        else orc_bonds(dim, L, seed, sweep, *thr, spins, open);
        if (orc_label_bfs(dim, L, open, lab) < 0) { rc = -1; break; }
        orc_flip(dim, L, seed, sweep, lab, spins);
        if (series) {
            if (mode & ORC_OPEN) orc_measure_open(dim, L, spins, &series[2 * k], &series[2 * k + 1]);
            else orc_measure(dim, L, spins, &series[2 * k], &series[2 * k + 1]);
        }
        if (mode & ORC_PCC) {
            int pc = (mode & ORC_OPEN) ? orc_spans_open(dim, L, lab)
                     : (mode & ORC_WIND) ? orc_winds(dim, L, open) : orc_percolates(dim, L, lab);
            if (pc < 0) { rc = -1; break; }
            if (perc) perc[k] = pc;
            orc_pcc_update(p, thr, pc, sweep, dp0, halve_every);
            if (p_trace) p_trace[k] = *p;
        }
    }
    if (!labels) free(lab);
    free(open);
    return rc;
}

int orc_run(int dim, int L, uint64_t seed, uint32_t s0, int32_t nsweeps,
            uint64_t *thr, double *p, int pcc, double dp0, uint32_t halve_every,
            int8_t *spins, int64_t *series, int32_t *labels, int32_t *perc, double *p_trace)
{
    if (orc_validate(dim, L) != 0 || nsweeps < 0) return -1;
    if (pcc && halve_every == 0) return -1;
    int64_t n = orc_nsites(dim, L);
    int32_t *lab = labels ? labels : (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!lab) return -1;
    int rc = 0;
    for (int32_t k = 0; k < nsweeps; ++k) {
        uint32_t sweep = s0 + (uint32_t)k;
        if (orc_sweep(dim, L, seed, sweep, *thr, spins, lab) != 0) { rc = -1; break; }
        if (series) orc_measure(dim, L, spins, &series[2 * k], &series[2 * k + 1]);
        if (pcc) {
            int pc = orc_percolates(dim, L, lab);
            if (pc < 0) { rc = -1; break; }
            if (perc) perc[k] = pc;
            orc_pcc_update(p, thr, pc, sweep, dp0, halve_every);
            if (p_trace) p_trace[k] = *p;
        }
    }
    if (!labels) free(lab);
    return rc;
}
