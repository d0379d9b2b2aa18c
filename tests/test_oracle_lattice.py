"""Pins of the oracle's bonds, labels, flip and observables (CPU only).

Labels are checked against scipy's connected components and a naive
union-find on the bond graph; the canonical label is the minimum site index
(Sec. II.B adopts the smaller label when clusters meet).  Special cases p=0
and p=1 reduce to the identity and to same-spin domains.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from paper_0808_2109_amd import workloads


def forward(dim, L, d):
    """Index of i + e_d for every site i (periodic)."""
    n = L ** dim
    idx = np.arange(n)
    stride = L ** d
    coord = (idx // stride) % L
    return np.where(coord == L - 1, idx - (L - 1) * stride, idx + stride)


def scipy_labels(dim, L, open_):
    n = L ** dim
    rows, cols = [], []
    for d in range(dim):
        f = forward(dim, L, d)
        sel = np.nonzero(open_[d])[0]
        rows.append(sel)
        cols.append(f[sel])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    g = coo_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    # canonical: minimum index per component
    mins = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


def naive_union_find(dim, L, open_):
    n = L ** dim
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for d in range(dim):
        f = forward(dim, L, d)
        for i in range(n):
            if open_[d][i]:
                a, b = find(i), find(int(f[i]))
                if a != b:
                    parent[max(a, b)] = min(a, b)
    return np.array([find(i) for i in range(n)], dtype=np.int32)


CASES = [(2, 3, 0.7), (2, 5, 0.3), (2, 8, 0.586), (2, 13, 0.9), (3, 3, 0.5), (3, 4, 0.36), (3, 6, 0.8)]


@pytest.mark.parametrize("dim,L,p", CASES)
def test_labels_match_scipy_and_union_find(orc, dim, L, p):
    thr = orc.threshold_from_p(p)
    for trial in range(3):
        seed = 100 + trial
        spins = workloads.random_spins(dim, L, seed)
        op = orc.bonds(dim, L, seed, trial, thr, spins)
        lab = orc.label_bfs(dim, L, op)
        assert np.array_equal(lab, scipy_labels(dim, L, op))
        if L ** dim <= 64:
            assert np.array_equal(lab, naive_union_find(dim, L, op))


@pytest.mark.parametrize("dim,L", [(2, 16), (3, 7)])
def test_label_invariants(orc, dim, L):
    thr = orc.threshold_from_p(0.6)
    spins = workloads.random_spins(dim, L, 7)
    op = orc.bonds(dim, L, 7, 0, thr, spins)
    lab = orc.label_bfs(dim, L, op)
    idx = np.arange(L ** dim)
    assert np.all(lab <= idx)
    assert np.array_equal(lab[lab], lab)
    for d in range(dim):
        f = forward(dim, L, d)
        sel = op[d].astype(bool)
        assert np.array_equal(lab[sel], lab[f[sel]])
        # bonds only between equal spins
        assert np.all(spins[sel] == spins[f[sel]])


def test_p_zero_every_site_alone(orc):
    for dim, L in [(2, 9), (3, 5)]:
        spins = workloads.random_spins(dim, L, 1)
        op = orc.bonds(dim, L, 1, 0, 0, spins)
        assert op.sum() == 0
        assert np.array_equal(orc.label_bfs(dim, L, op), np.arange(L ** dim, dtype=np.int32))


def test_p_one_uniform_spins_one_cluster(orc):
    for dim, L in [(2, 9), (3, 5)]:
        spins = np.ones(L ** dim, dtype=np.int8)
        op = orc.bonds(dim, L, 1, 0, 2**32, spins)
        assert op.all()
        assert np.all(orc.label_bfs(dim, L, op) == 0)


def test_p_one_random_spins_gives_same_spin_domains(orc):
    for dim, L in [(2, 11), (3, 6)]:
        spins = workloads.random_spins(dim, L, 4)
        op = orc.bonds(dim, L, 4, 2, 2**32, spins)
        equal = np.stack([spins == spins[forward(dim, L, d)] for d in range(dim)]).astype(np.uint8)
        assert np.array_equal(op, equal)
        assert np.array_equal(orc.label_bfs(dim, L, op), scipy_labels(dim, L, equal))


@pytest.mark.parametrize("dim,L", [(2, 12), (3, 5)])
def test_flip_gives_each_cluster_one_fresh_spin(orc, dim, L):
    seed, sweep = 21, 4
    thr = orc.threshold_from_p(0.55)
    spins = workloads.random_spins(dim, L, seed)
    new, lab = orc.sweep(dim, L, seed, sweep, thr, spins)
    for r in np.unique(lab):
        members = new[lab == r]
        assert np.all(members == members[0])
        assert members[0] == orc.flip_spin(seed, sweep, int(r))


def test_p_zero_sweep_is_iid_redraw(orc):
    dim, L = 2, 64
    spins = workloads.random_spins(dim, L, 2)
    new, lab = orc.sweep(dim, L, 2, 9, 0, spins)
    assert np.array_equal(lab, np.arange(L * L, dtype=np.int32))
    assert abs(int(new.astype(np.int64).sum())) < 5 * 64
    assert np.array_equal(new, orc.flip(dim, L, 2, 9, np.arange(L * L, dtype=np.int32)))


def numpy_measure(dim, L, spins):
    s = spins.astype(np.int64).reshape((L,) * dim)
    e = 0
    for ax in range(dim):
        e += int((s * np.roll(s, -1, axis=dim - 1 - ax)).sum())
    return e, int(s.sum())


@pytest.mark.parametrize("dim,L", [(2, 4), (2, 10), (3, 4), (3, 7)])
def test_measure(orc, dim, L):
    n = L ** dim
    up = np.ones(n, dtype=np.int8)
    assert orc.measure(dim, L, up) == (dim * n, n)
    assert orc.measure(dim, L, -up) == (dim * n, -n)
    if L % 2 == 0:
        coords = np.indices((L,) * dim).sum(axis=0).reshape(-1)
        cb = np.where(coords % 2 == 0, 1, -1).astype(np.int8)
        assert orc.measure(dim, L, cb) == (-dim * n, 0)
    rnd = workloads.random_spins(dim, L, 5)
    assert orc.measure(dim, L, rnd) == numpy_measure(dim, L, rnd)


def test_validate(orc):
    assert orc.validate(2, 3)
    assert not orc.validate(2, 2)
    assert not orc.validate(4, 10)
    assert orc.validate(2, 46340)
    assert not orc.validate(2, 46341)          # N >= 2^31
    assert orc.validate(3, 1127)              # 3 N < 2^32 (link indices are 32-bit)
    assert not orc.validate(3, 1128)


def test_run_matches_step_by_step(orc):
    dim, L, seed = 2, 10, 77
    thr = orc.threshold(1.0, 2.3)
    res = orc.run(dim, L, seed, 5, thr=thr)
    s = orc.init_spins(dim, L, seed)
    for k in range(5):
        s, lab = orc.sweep(dim, L, seed, k, thr, s)
        assert tuple(res["series"][k]) == orc.measure(dim, L, s)
    assert np.array_equal(res["spins"], s)
    assert np.array_equal(res["labels"], lab)
    # resuming from a saved state continues the same chain
    head = orc.run(dim, L, seed, 2, thr=thr)
    tail = orc.run(dim, L, seed, 3, thr=thr, s0=2, spins=head["spins"])
    assert np.array_equal(tail["spins"], res["spins"])
