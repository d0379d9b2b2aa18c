"""Pins of the oracle's whole Markov chain against exact Ising results (CPU).

The chain is stochastic, so these are statistical tests: sample means of the
oracle's per-sweep series are compared with exact expectations at 5 standard
errors (batch-means errors), and the sampled energy histogram of the 4x4
torus with its exact distribution (chi-square).  A dropped term, a wrong sign
or a wrong bond probability moves these averages by many standard errors.

Exact values come from brute-force enumeration (4x4), a layer transfer matrix
(3x3x3), Kaufman's finite-torus partition function (L = 16), Onsager's T_c and
Yang's magnetisation; see tests/exact.py.
"""
import math

import numpy as np
import pytest

import exact

TC = exact.TC_2D


def batch_mean_err(x, nbatch=50):
    x = np.asarray(x, dtype=np.float64)
    n = (x.size // nbatch) * nbatch
    b = x[:n].reshape(nbatch, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbatch))


def chain(orc, dim, L, T, sweeps, seed, burn=200):
    res = orc.run(dim, L, seed, sweeps + burn, T=T, keep_labels=False)
    series = res["series"][burn:]
    n = L ** dim
    e = -series[:, 0] / n
    m = np.abs(series[:, 1]) / n
    return e, m, series


def test_enumeration_matches_known_degeneracies():
    hist = exact.histogram_2d(4)
    g = {}
    for (e, _m), c in hist.items():
        g[e] = g.get(e, 0) + c
    assert sum(g.values()) == 2 ** 16
    assert g[32] == g[-32] == 2
    assert g[0] == 20524
    assert g[24] == 32


@pytest.mark.parametrize("T", [TC, 2.0, 3.0])
def test_4x4_chain_matches_enumeration(orc, T):
    hist = exact.histogram_2d(4)
    ex = exact.averages_from_histogram(hist, 16, T)
    e, m, series = chain(orc, 2, 4, T, 200000, seed=11)
    em, ee = batch_mean_err(e)
    mm, me = batch_mean_err(m)
    assert abs(em - ex["e"]) < 5 * ee, (em, ex["e"], ee)
    assert abs(mm - ex["abs_m"]) < 5 * me, (mm, ex["abs_m"], me)
    # histogram of E_int against exp(K E) g(E) / Z
    es, prob = exact.energy_distribution(hist, T)
    counts = np.array([(series[:, 0] == v).sum() for v in es], dtype=np.float64)
    assert counts.sum() == series.shape[0]
    expct = prob * series.shape[0]
    keep = expct > 20
    chi2 = float((((counts - expct) ** 2 / expct)[keep]).sum())
    dof = int(keep.sum()) - 1
    # SW samples are mildly correlated; allow a generous margin over dof
    assert chi2 < 3.0 * dof + 30, (chi2, dof)


def test_3x3x3_chain_matches_transfer_matrix(orc):
    T = 4.5115
    ex = exact.cube3_averages(T)
    assert abs(ex["Z_check"] - 1.0) < 1e-9
    e, m, _ = chain(orc, 3, 3, T, 150000, seed=5)
    em, ee = batch_mean_err(e)
    mm, me = batch_mean_err(m)
    assert abs(em - ex["e"]) < 5 * ee, (em, ex["e"], ee)
    assert abs(mm - ex["abs_m"]) < 5 * me, (mm, ex["abs_m"], me)


def test_transfer_matrix_matches_brute_force_sum():
    # pins the pin: the 3x3x3 transfer matrix energy at high T expands as -3K + O(K^3)
    T = 1000.0
    ex = exact.cube3_averages(T)
    assert abs(ex["e"] - (-3.0 / T)) < 1e-4


def test_kaufman_matches_enumeration_4x4():
    hist = exact.histogram_2d(4)
    for T in (TC, 2.0, 3.0):
        ex = exact.averages_from_histogram(hist, 16, T)
        assert abs(exact.kaufman_energy(4, T) - ex["e"]) < 1e-10
        import mpmath as mp

        assert abs(float(exact.kaufman_lnZ(mp.mpf(1) / T, 4, 4)) - ex["lnZ"]) < 1e-10


def test_kaufman_approaches_onsager_at_tc():
    # e(T_c, L) -> -sqrt(2) as L grows (Onsager)
    e64 = exact.kaufman_energy(64, TC)
    e128 = exact.kaufman_energy(128, TC)
    assert abs(e128 + math.sqrt(2)) < abs(e64 + math.sqrt(2)) < 0.02
    assert abs((e64 + math.sqrt(2)) * 64 - (e128 + math.sqrt(2)) * 128) < 0.01


def test_16x16_chain_matches_kaufman_at_tc(orc):
    ex = exact.kaufman_energy(16, TC)
    e, _m, _ = chain(orc, 2, 16, TC, 60000, seed=3)
    em, ee = batch_mean_err(e)
    assert abs(em - ex) < 5 * ee, (em, ex, ee)
    assert ee < 0.004


def test_32x32_magnetisation_near_yang_at_T2(orc):
    # deep in the ordered phase finite-size corrections are small
    _e, m, _ = chain(orc, 2, 32, 2.0, 4000, seed=9)
    mm, me = batch_mean_err(m, nbatch=20)
    assert abs(mm - exact.yang_magnetisation(2.0)) < 0.01 + 5 * me
