"""Pins of the oracle's open boundaries and of its two other percolation tests
(Sec. III: the spanning test of an open box, the topological rule) (CPU only).

* Open boundaries: the bonds are the periodic ones (pinned elsewhere) with the
  links that would wrap removed; labels equal scipy's connected components of
  the open bond graph; E_int of a uniform state counts the links of the box;
  the whole chain on the open 4x4 box matches exact enumeration.
* Spanning of an open box: constructed cases, and scipy components checked for
  a cluster that holds sites of both opposite faces.
* Winding: constructed rings, spans that do not wind, windings along y, z and
  a diagonal, and on random bond sets an independent criterion: a cluster
  winds along axis a exactly when its preimage in the 7-fold cover of the
  torus along a (7 L sites along a, the same bonds repeated) is connected
  (on these small lattices no loop winds 7 times, so a winding cluster's
  preimage is one component and a non-winding one's is seven).
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import exact


def coords(dim, L):
    idx = np.arange(L ** dim)
    return [(idx // L ** d) % L for d in range(dim)]


def forward(dim, L, d):
    idx = np.arange(L ** dim)
    stride = L ** d
    c = (idx // stride) % L
    return np.where(c == L - 1, idx - (L - 1) * stride, idx + stride)


def scipy_min_labels(dim, L, open_):
    n = L ** dim
    rows, cols = [], []
    for d in range(dim):
        sel = np.nonzero(open_[d])[0]
        rows.append(sel)
        cols.append(forward(dim, L, d)[sel])
    g = coo_matrix((np.ones(sum(r.size for r in rows)), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    mins = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


@pytest.mark.parametrize("dim,L,p", [(2, 9, 0.6), (2, 16, 0.9), (3, 5, 0.5), (3, 7, 0.3)])
def test_open_bonds_are_the_periodic_ones_without_the_wrap(orc, dim, L, p):
    rng = np.random.default_rng(L)
    spins = np.where(rng.random(L ** dim) < 0.5, 1, -1).astype(np.int8)
    thr = orc.threshold_from_p(p)
    per = orc.bonds(dim, L, 7, 3, thr, spins)
    opn = orc.bonds_open(dim, L, 7, 3, thr, spins)
    for d, c in enumerate(coords(dim, L)):
        wrap = c == L - 1
        assert not opn[d][wrap].any()
        assert np.array_equal(opn[d][~wrap], per[d][~wrap])
    lab = orc.label_bfs(dim, L, opn)
    assert np.array_equal(lab, scipy_min_labels(dim, L, opn))


@pytest.mark.parametrize("dim,L", [(2, 6), (3, 4)])
def test_open_measure_counts_the_links_of_the_box(orc, dim, L):
    up = np.ones(L ** dim, dtype=np.int8)
    assert orc.measure_open(dim, L, up) == (dim * L ** (dim - 1) * (L - 1), L ** dim)
    # a checkerboard has every link unequal
    ch = np.where(sum(coords(dim, L)) % 2 == 0, 1, -1).astype(np.int8)
    e, m = orc.measure_open(dim, L, ch)
    assert e == -dim * L ** (dim - 1) * (L - 1)


def test_open_p_one_uniform_is_one_cluster(orc):
    dim, L = 2, 12
    up = np.ones(L * L, dtype=np.int8)
    opn = orc.bonds_open(dim, L, 1, 0, 2 ** 32, up)
    assert opn.sum() == 2 * L * (L - 1)
    assert not orc.label_bfs(dim, L, opn).any()


@pytest.mark.parametrize("T", [exact.TC_2D, 2.0])
def test_open_4x4_chain_matches_enumeration(orc, T):
    hist = exact.histogram_2d_open(4)
    ex = exact.averages_from_histogram(hist, 16, T)
    res = orc.run(2, 4, 21, 150200, T=T, keep_labels=False, open_bc=True)
    series = res["series"][200:]
    e = -series[:, 0] / 16.0
    m = np.abs(series[:, 1]) / 16.0
    for x, want in ((e, ex["e"]), (m, ex["abs_m"])):
        b = x[: (x.size // 50) * 50].reshape(50, -1).mean(axis=1)
        mean, err = b.mean(), b.std(ddof=1) / math.sqrt(50)
        assert abs(mean - want) < 5 * err, (mean, want, err)
    # the periodic value differs: the open box is really sampled
    per = exact.averages_from_histogram(exact.histogram_2d(4), 16, T)
    assert abs(per["e"] - ex["e"]) > 0.05


def _line(dim, L, axis, at, length, wrap):
    """Bonds of one straight line of `length` links along `axis` from the site
    `at`, including the wrap link when the line reaches coordinate L-1."""
    n = L ** dim
    opn = np.zeros((dim, n), dtype=np.uint8)
    stride = L ** axis
    i = at
    for _ in range(length):
        c = (i // stride) % L
        if c == L - 1 and not wrap:
            break
        opn[axis][i] = 1
        i = i - (L - 1) * stride if c == L - 1 else i + stride
    return opn


def test_open_spanning_constructed(orc):
    L = 8
    full = _line(2, L, 0, 3 * L, L - 1, wrap=False)           # row y = 3 from x = 0 to x = L-1
    lab = orc.label_bfs(2, L, full)
    assert orc.spans_open(2, L, lab)
    short = full.copy()
    short[0][3 * L + 4] = 0                                    # one link missing in the middle
    assert not orc.spans_open(2, L, orc.label_bfs(2, L, short))
    col = _line(2, L, 1, 5, L - 1, wrap=False)                 # column x = 5 spans y
    assert orc.spans_open(2, L, orc.label_bfs(2, L, col))
    assert not orc.spans_open(2, L, np.arange(L * L, dtype=np.int32))
    L3 = 5
    zl = _line(3, L3, 2, 7, L3 - 1, wrap=False)
    assert orc.spans_open(3, L3, orc.label_bfs(3, L3, zl))


# spins mostly up, so that the bond graph sits near its percolation point and
# both outcomes occur
@pytest.mark.parametrize("dim,L,p", [(2, 8, 0.45), (2, 8, 0.5), (2, 12, 0.55), (3, 5, 0.2), (3, 6, 0.22)])
def test_open_spanning_matches_components(orc, dim, L, p):
    rng = np.random.default_rng(17 * L + dim)
    thr = orc.threshold_from_p(p)
    hits = 0
    for k in range(20):
        spins = np.where(rng.random(L ** dim) < 0.9, 1, -1).astype(np.int8)
        opn = orc.bonds_open(dim, L, 5, k, thr, spins)
        lab = scipy_min_labels(dim, L, opn)
        want = any(np.intersect1d(lab[c == 0], lab[c == L - 1]).size > 0 for c in coords(dim, L))
        assert orc.spans_open(dim, L, lab) == want
        hits += want
    assert 0 < hits < 20


def test_winding_constructed(orc):
    L = 7
    ring = _line(2, L, 0, 2 * L, L, wrap=True)                 # row y = 2 closed around the box
    assert orc.winds(2, L, ring)
    assert orc.percolates(2, L, orc.label_bfs(2, L, ring))
    open_row = _line(2, L, 0, 2 * L, L, wrap=False)            # the same row without its wrap link
    assert not orc.winds(2, L, open_row)
    assert orc.percolates(2, L, orc.label_bfs(2, L, open_row))   # spans (extension rule) but does not wind
    yring = _line(2, L, 1, 4, L, wrap=True)
    assert orc.winds(2, L, yring)
    # a staircase around the diagonal: x-link then y-link, L times: winding (1, 1)
    stair = np.zeros((2, L * L), dtype=np.uint8)
    x = y = 0
    for _ in range(L):
        stair[0][x + L * y] = 1
        x = (x + 1) % L
        stair[1][x + L * y] = 1
        y = (y + 1) % L
    assert orc.winds(2, L, stair)
    # a contractible loop (a 2x2 plaquette) does not wind
    sq = np.zeros((2, L * L), dtype=np.uint8)
    sq[0][0] = sq[0][L] = sq[1][0] = sq[1][1] = 1
    assert not orc.winds(2, L, sq)
    L3 = 4
    assert orc.winds(3, L3, _line(3, L3, 2, 5, L3, wrap=True))
    assert not orc.winds(3, L3, _line(3, L3, 2, 5, L3, wrap=False))


def _cover_components(dim, L, opn, cluster_sites, axis, m=7):
    """Components of the preimage of a cluster in the m-fold cover along axis."""
    shape = [L] * dim
    shape[axis] = m * L
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[:d])) for d in range(dim)]
    idx = np.arange(n)
    cc = [(idx // strides[d]) % shape[d] for d in range(dim)]
    base = sum((cc[d] % L) * L ** d for d in range(dim))           # the site of the box each cover site sits over
    rows, cols = [], []
    for d in range(dim):
        sel = np.nonzero(opn[d][base])[0]
        nxt = np.where(cc[d][sel] == shape[d] - 1, sel - (shape[d] - 1) * strides[d], sel + strides[d])
        rows.append(sel)
        cols.append(nxt)
    g = coo_matrix((np.ones(sum(r.size for r in rows)), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    members = np.isin(base, cluster_sites)
    return np.unique(comp[members]).size


@pytest.mark.parametrize("dim,L,p", [(2, 5, 0.5), (2, 5, 0.6), (2, 6, 0.55), (3, 4, 0.25), (3, 4, 0.32)])
def test_winding_matches_the_cover_criterion(orc, dim, L, p):
    rng = np.random.default_rng(31 * L + dim)
    thr = orc.threshold_from_p(p)
    seen = [0, 0]
    for k in range(25):
        spins = np.where(rng.random(L ** dim) < 0.9, 1, -1).astype(np.int8)
        opn = orc.bonds(dim, L, 9, k, thr, spins)
        lab = orc.label_bfs(dim, L, opn)
        want = False
        for r in np.unique(lab):
            sites = np.nonzero(lab == r)[0]
            if sites.size < L:
                continue
            for axis in range(dim):
                if _cover_components(dim, L, opn, sites, axis) < 7:
                    want = True
        got = orc.winds(dim, L, opn)
        assert got == want, k
        if got:
            assert orc.percolates(dim, L, lab)                    # a winding cluster spans that axis
        seen[got] += 1
    assert seen[0] and seen[1]


@pytest.mark.parametrize("open_bc,wind", [(True, False), (False, True)])
def test_pcc_runs_follow_their_rule(orc, open_bc, wind):
    dim, L, seed, n = 2, 12, 4, 60
    res = orc.run(dim, L, seed, n, p=0.5, pcc=True, open_bc=open_bc, wind=wind, dp0=0.02, halve_every=15)
    spins = orc.init_spins(dim, L, seed)
    p, thr = 0.5, orc.threshold_from_p(0.5)
    for k in range(n):
        opn = (orc.bonds_open if open_bc else orc.bonds)(dim, L, seed, k, thr, spins)
        lab = orc.label_bfs(dim, L, opn)
        spins = orc.flip(dim, L, seed, k, lab)
        flag = orc.spans_open(dim, L, lab) if open_bc else orc.winds(dim, L, opn)
        assert bool(res["perc"][k]) == flag, k
        p, thr = orc.pcc_update(p, thr, flag, k, dp0=0.02, halve_every=15)
        assert res["p_trace"][k] == p
    assert np.array_equal(res["spins"], spins)
    assert 0 < res["perc"].sum() < n
