"""Pins of the oracle's percolation test and PCC feedback (CPU only).

* The range operator of Sec. III reproduces the paper's worked example
  (tests/golden/pcc_range_example.json).
* The oracle's coordinate-set test agrees with the interval form on the
  clusters of real sweeps, and with constructed spanning / non-spanning cases.
* The feedback law p -/+ dp with dp halved every `halve_every` sweeps and
  clamping to [0, 1].
"""
import json
import os

import numpy as np
import pytest

from oracle import ranges
from paper_0808_2109_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pcc_range_example.json")


def test_worked_example_of_range_merge():
    ex = json.load(open(GOLDEN))
    c1 = [tuple(t) for t in ex["before"]["cluster_1"]]
    c8 = [tuple(t) for t in ex["before"]["cluster_8"]]
    merged = ranges.merge(c1, c8)
    assert merged == [tuple(t) for t in ex["after_merge"]["cluster_1"]]
    assert ranges.covers(merged, ex["L"]) == ex["percolating"]
    # one more site at x = 4 would close the gap and make the cluster span
    assert ranges.covers(ranges.merge(merged, [(4, 4)]), ex["L"])


def test_worked_example_as_lattice(orc):
    # a 16 x 3 strip is not a valid periodic lattice (L is per axis), so embed
    # the example in a 16 x 16 lattice: cluster 1 occupies x in [0,3] u [5,15]
    # on row 0, every other site is its own cluster.
    L = 16
    lab = np.arange(L * L, dtype=np.int32)
    row0 = [x for x in range(16) if x != 4]
    lab[row0] = 0
    assert not orc.percolates(2, L, lab)
    assert not ranges.percolates(lab, 2, L)
    lab[4] = 0
    assert orc.percolates(2, L, lab)
    assert ranges.percolates(lab, 2, L)


@pytest.mark.parametrize("dim,L,p", [(2, 8, 0.4), (2, 8, 0.6), (2, 12, 0.586), (3, 5, 0.3), (3, 6, 0.45)])
def test_coordinate_sets_agree_with_ranges(orc, dim, L, p):
    thr = orc.threshold_from_p(p)
    seen = set()
    for trial in range(6):
        spins = workloads.random_spins(dim, L, 40 + trial)
        _, lab = orc.sweep(dim, L, 40 + trial, trial, thr, spins)
        a = orc.percolates(dim, L, lab)
        assert a == ranges.percolates(lab, dim, L)
        seen.add(a)
    # the chosen p values near the threshold produce both outcomes across cases
    assert seen


def test_constructed_cases(orc):
    L = 10
    # p = 1, all up: one cluster spans every axis
    lab = np.zeros(L * L, dtype=np.int32)
    assert orc.percolates(2, L, lab)
    # all sites alone: no cluster spans (L >= 2)
    assert not orc.percolates(2, L, np.arange(L * L, dtype=np.int32))
    # one full column spans y but not x
    lab = np.arange(L * L, dtype=np.int32)
    col = np.arange(L) * L + 3
    lab[col] = 3
    assert orc.percolates(2, L, lab)
    # a diagonal staircase covers every x and every y
    lab = np.arange(L * L, dtype=np.int32)
    diag = np.arange(L) * L + np.arange(L)
    lab[diag] = 0
    assert orc.percolates(2, L, lab)
    # a 3D plane z = 2 spans x and y
    L3 = 5
    lab = np.arange(L3 ** 3, dtype=np.int32)
    plane = np.arange(L3 * L3) + 2 * L3 * L3
    lab[plane] = plane[0]
    assert orc.percolates(3, L3, lab)


def test_feedback_law(orc):
    p, thr = orc.pcc_update(0.5, 2**31, True, 0)
    assert p == 0.49 and thr == orc.threshold_from_p(0.49)
    p, _ = orc.pcc_update(0.5, 2**31, False, 999)
    assert p == 0.51
    p, _ = orc.pcc_update(0.5, 2**31, False, 1000)
    assert p == 0.5 + 0.005
    p, _ = orc.pcc_update(0.5, 2**31, True, 2500)
    assert p == 0.5 - 0.0025
    p, thr = orc.pcc_update(0.995, 0, False, 0)
    assert p == 1.0 and thr == 2**32
    p, thr = orc.pcc_update(0.004, 0, True, 0)
    assert p == 0.0 and thr == 0
    p, _ = orc.pcc_update(0.5, 0, False, 3, dp0=0.02, halve_every=2)
    assert p == 0.5 + 0.01


def test_pcc_run_follows_its_percolation_flags(orc):
    dim, L = 2, 16
    res = orc.run(dim, L, 3, 400, p=0.5, pcc=True)
    p = 0.5
    for k in range(400):
        p, _ = orc.pcc_update(p, 0, bool(res["perc"][k]), k)
        assert res["p_trace"][k] == p
    assert res["p"] == p
    # feedback drives p towards the percolation threshold (2 - sqrt 2 in the
    # thermodynamic limit); at L = 16 it settles in a broad window around it
    assert 0.45 < float(np.mean(res["p_trace"][200:])) < 0.7
