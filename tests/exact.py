"""Exact Ising results used to pin the oracle (test helpers, no oracle code).

* brute-force enumeration of small periodic lattices (joint histogram of
  E_int = sum over links s_i s_j and M = sum s_i);
* a layer transfer matrix for the 3x3x3 periodic cube;
* Kaufman's exact partition function of the finite periodic square lattice
  (B. Kaufman, Phys. Rev. 76, 1232 (1949); in the form of A. E. Ferdinand and
  M. E. Fisher, Phys. Rev. 185, 832 (1969)), with the energy by numerical
  differentiation of ln Z in K = J/T;
* Onsager's critical temperature and Yang's spontaneous magnetisation.
"""
from __future__ import annotations

import math

import numpy as np

TC_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))


def _bits(states: np.ndarray, n: int) -> np.ndarray:
    return ((states[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int8) * 2 - 1


def histogram_2d(L: int):
    """Joint histogram {(E_int, M): count} of the L x L periodic lattice (L <= 5)."""
    n = L * L
    states = np.arange(1 << n, dtype=np.int64)
    s = _bits(states, n).reshape(-1, L, L)          # [state, y, x]
    e = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) + (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    m = s.sum(axis=(1, 2))
    keys, counts = np.unique(np.stack([e, m], axis=1), axis=0, return_counts=True)
    return {(int(a), int(b)): int(c) for (a, b), c in zip(keys, counts)}


def averages_from_histogram(hist: dict, n: int, T: float, J: float = 1.0):
    """<e> = <-J E_int>/N, <|m|> = <|M|>/N, <m^2>, and ln Z at temperature T."""
    K = J / T
    es = np.array([k[0] for k in hist], dtype=np.float64)
    ms = np.array([k[1] for k in hist], dtype=np.float64)
    g = np.array(list(hist.values()), dtype=np.float64)
    w = g * np.exp(K * (es - es.max()))
    z = w.sum()
    return {
        "e": float((-J * es * w).sum() / z / n),
        "abs_m": float((np.abs(ms) * w).sum() / z / n),
        "m2": float((ms * ms * w).sum() / z / n / n),
        "lnZ": float(math.log(z) + K * es.max()),
    }


def energy_distribution(hist: dict, T: float, J: float = 1.0):
    """Exact probability of every E_int value."""
    K = J / T
    per_e: dict = {}
    for (e, _m), c in hist.items():
        per_e[e] = per_e.get(e, 0) + c
    es = np.array(sorted(per_e), dtype=np.int64)
    g = np.array([per_e[e] for e in es], dtype=np.float64)
    w = g * np.exp(K * (es - es.max()))
    return es, w / w.sum()


def cube3_averages(T: float, J: float = 1.0):
    """Exact <e>, <|m|> of the 3x3x3 periodic simple-cubic Ising model.

    The cube is three periodic 3x3 layers; the transfer matrix between layer
    states a, b carries half of each layer's in-plane energy, the inter-layer
    energy, and z^((M_a + M_b)/2) for the magnetisation.  Tr(T^3) as a
    polynomial in z is recovered from its values on roots of unity.
    """
    K = J / T
    layer = _bits(np.arange(512, dtype=np.int64), 9).reshape(512, 3, 3)
    e_in = (layer * np.roll(layer, -1, axis=2)).sum(axis=(1, 2)) + (layer * np.roll(layer, -1, axis=1)).sum(axis=(1, 2))
    m_l = layer.sum(axis=(1, 2)).astype(np.float64)
    e_ab = np.einsum("ayx,byx->ab", layer.astype(np.float64), layer.astype(np.float64))
    ework = 0.5 * e_in[:, None] + 0.5 * e_in[None, :] + e_ab    # E_int shared per transfer step
    shift = 27.0 * 3.0 / 3.0                                     # keep exponents small
    base = np.exp(K * (ework - shift))
    # moments of energy: Z = Tr(B^3), dZ/dK = 3 Tr(B^2 (B*E)) (+ the shift term)
    b2 = base @ base
    z = np.trace(b2 @ base)
    dz = 3.0 * np.trace(b2 @ (base * (ework - shift)))
    e_mean_int = dz / z + 3.0 * shift                             # <E_int>
    # magnetisation distribution via z-transform on 28 roots of unity (M in -27..27 step 2)
    nroot = 64
    coeffs = np.zeros(nroot, dtype=np.complex128)
    for k in range(nroot):
        w = np.exp(2j * np.pi * k / nroot)
        phase = w ** (0.5 * (m_l[:, None] + m_l[None, :]))
        bz = base * phase
        coeffs[k] = np.trace(bz @ bz @ bz)
    # Tr(B(z)^3) = sum_M Z_M z^M ; M odd in [-27, 27]; invert the DFT
    zm = {}
    for M in range(-27, 28, 2):
        val = sum(coeffs[k] * np.exp(-2j * np.pi * k * M / nroot) for k in range(nroot)) / nroot
        zm[M] = val.real
    ztot = sum(zm.values())
    abs_m = sum(abs(M) * v for M, v in zm.items()) / ztot / 27.0
    return {"e": float(-J * e_mean_int / 27.0), "abs_m": float(abs_m), "Z_check": float(ztot / z)}


def kaufman_lnZ(K, m: int, n: int):
    """ln Z of the m x n periodic square lattice at coupling K (mpmath value).

    Z = 1/2 (2 sinh 2K)^(mn/2) * sum_{i=1..4} Z_i with
      Z1 = prod_r 2 cosh(m g_{2r+1}/2), Z2 = prod_r 2 sinh(m g_{2r+1}/2),
      Z3 = prod_r 2 cosh(m g_{2r}/2),   Z4 = prod_r 2 sinh(m g_{2r}/2),
    r = 0..n-1, cosh g_l = cosh 2K coth 2K - cos(pi l / n) for l > 0 and the
    signed g_0 = 2K + ln tanh K.
    """
    import mpmath as mp

    K = mp.mpf(K)

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(mp.cosh(2 * K) * mp.coth(2 * K) - mp.cos(mp.pi * l / n))

    z1 = z2 = z3 = z4 = mp.mpf(1)
    for r in range(n):
        go = gamma(2 * r + 1)
        ge = gamma(2 * r)
        z1 *= 2 * mp.cosh(m * go / 2)
        z2 *= 2 * mp.sinh(m * go / 2)
        z3 *= 2 * mp.cosh(m * ge / 2)
        z4 *= 2 * mp.sinh(m * ge / 2)
    return mp.log(mp.mpf(1) / 2) + (m * n / mp.mpf(2)) * mp.log(2 * mp.sinh(2 * K)) + mp.log(z1 + z2 + z3 + z4)


def kaufman_energy(L: int, T: float, J: float = 1.0, digits: int = 40) -> float:
    """Exact <e> = -J <E_int>/N of the L x L torus: -(1/N) d lnZ/dK * J."""
    import mpmath as mp

    with mp.workdps(digits):
        K = mp.mpf(J) / mp.mpf(T)
        dlnz = mp.diff(lambda k: kaufman_lnZ(k, L, L), K)
        return float(-J * dlnz / (L * L))


def yang_magnetisation(T: float, J: float = 1.0) -> float:
    """Spontaneous magnetisation of the infinite square lattice (C. N. Yang, 1952)."""
    return (1.0 - math.sinh(2.0 * J / T) ** -4) ** 0.125


def histogram_2d_open(L: int):
    """Joint histogram {(E_int, M): count} of the L x L lattice with open
    boundaries (only the 2 L (L - 1) links inside the box), L <= 5."""
    n = L * L
    states = np.arange(1 << n, dtype=np.int64)
    s = _bits(states, n).reshape(-1, L, L)          # [state, y, x]
    e = (s[:, :, :-1] * s[:, :, 1:]).sum(axis=(1, 2)) + (s[:, :-1, :] * s[:, 1:, :]).sum(axis=(1, 2))
    m = s.sum(axis=(1, 2))
    keys, counts = np.unique(np.stack([e, m], axis=1), axis=0, return_counts=True)
    return {(int(a), int(b)): int(c) for (a, b), c in zip(keys, counts)}
