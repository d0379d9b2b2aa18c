"""Pins of the oracle's random stream and bond threshold (CPU only).

* Philox4x32-10 against two independent implementations of the SC'11
  generator that ship as source headers here: ATen's PhiloxRNGEngine.h
  (compiled with g++) and rocRAND's rocrand_philox4x32_10.h (host-compiled
  with hipcc).
* The bond probability P = 1 - exp(-2J/T) (Sec. I, step 1) against its closed
  form at the 2D critical point, P(T_c) = 2 - sqrt(2), and against 50-digit
  evaluation.
* The two-stage bond decision against the plain definition u < thr with
  u = a * 2^24 + b, and against its binomial statistics.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
TORCH_INC = None
try:
    import torch  # noqa: F401

    TORCH_INC = os.path.join(os.path.dirname(torch.__file__), "include")
except Exception:  # pragma: no cover
    TORCH_INC = None


def _random_blocks(n, seed):
    rng = np.random.default_rng(seed)
    words = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64)
    # include structured counters like the ones the method uses
    words[: n // 4, 1] = 0
    words[: n // 4, 3] = rng.integers(0, 4, size=n // 4)
    words[0] = 0
    words[1] = 2**32 - 1
    return words


def _run_xcheck(exe, blocks):
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in blocks) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def _oracle_blocks(orc, blocks):
    return np.array([orc.philox(row[:4], row[4:]) for row in blocks], dtype=np.uint64)


@pytest.mark.skipif(TORCH_INC is None or shutil.which("g++") is None, reason="needs torch headers and g++")
def test_philox_matches_aten(orc, tmp_path):
    exe = str(tmp_path / "philox_aten")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I" + TORCH_INC, "-o", exe,
                           os.path.join(HERE, "xcheck", "philox_aten.cpp")])
    blocks = _random_blocks(3000, 11)
    assert np.array_equal(_run_xcheck(exe, blocks), _oracle_blocks(orc, blocks))


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists("/opt/rocm/include/rocrand"),
                    reason="needs hipcc and rocRAND headers")
def test_philox_matches_rocrand(orc, tmp_path):
    exe = str(tmp_path / "philox_rocrand")
    subprocess.check_call(["hipcc", "-O1", "-o", exe, os.path.join(HERE, "xcheck", "philox_rocrand.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    blocks = _random_blocks(3000, 12)
    assert np.array_equal(_run_xcheck(exe, blocks), _oracle_blocks(orc, blocks))


def test_threshold_closed_form_at_tc(orc):
    import mpmath as mp

    tc = 2.0 / math.log(1.0 + math.sqrt(2.0))
    # 1 - exp(-2/T_c) = 1 - 1/(1 + sqrt 2) = 2 - sqrt 2 exactly
    with mp.workdps(60):
        exact = mp.floor((2 - mp.sqrt(2)) * mp.mpf(2) ** 32)
    assert orc.threshold(1.0, tc) == int(exact) == 2515933592
    assert abs(orc.bond_probability(1.0, tc) - (2.0 - math.sqrt(2.0))) < 1e-15


@pytest.mark.parametrize("J,T", [(1.0, 2.0), (1.0, 2.6), (1.0, 4.5115), (0.5, 1.3), (1.0, 0.2), (2.0, 100.0)])
def test_threshold_matches_high_precision(orc, J, T):
    import mpmath as mp

    with mp.workdps(60):
        exact = (1 - mp.exp(-2 * mp.mpf(J) / mp.mpf(T))) * mp.mpf(2) ** 32
        frac = exact - mp.floor(exact)
    # the double evaluation may only differ from the exact floor next to an integer
    assert min(frac, 1 - frac) > 1e-4
    assert orc.threshold(J, T) == int(mp.floor(exact))


def test_threshold_edges(orc):
    assert orc.threshold_from_p(0.0) == 0
    assert orc.threshold_from_p(-0.5) == 0
    assert orc.threshold_from_p(1.0) == 2**32
    assert orc.threshold_from_p(0.5) == 2**31
    assert orc.threshold_from_p(float(np.nextafter(1.0, 0.0))) == 2**32 - 1


def _u32(orc, seed, sweep, link):
    """The uniform 32-bit u = a * 2^24 + b that the bond decision compares."""
    k = link & 15
    blk = orc.philox([link >> 4, 0, sweep, 1], [seed & 0xFFFFFFFF, seed >> 32])
    a = (int(blk[k >> 2]) >> (8 * (k & 3))) & 0xFF
    ref = orc.philox([link >> 2, 0, sweep, 2], [seed & 0xFFFFFFFF, seed >> 32])
    b = int(ref[link & 3]) & 0xFFFFFF
    return (a << 24) | b


def test_two_stage_bond_equals_single_compare(orc):
    rng = np.random.default_rng(3)
    seed, sweep = 0x1234_5678_9ABC, 17
    links = rng.integers(0, 2**32, size=600).tolist() + list(range(64))
    for link in links:
        u = _u32(orc, seed, sweep, link)
        # thresholds that tie on the high byte exercise the refinement path
        for thr in (u, u + 1, max(u - 1, 0), (u & 0xFF000000) | 0x00800000, 0, 2**32, 2515933592):
            assert orc.bond_open(seed, sweep, thr, link, True) == int(u < thr), (link, thr)
            assert orc.bond_open(seed, sweep, thr, link, False) == 0


def test_bond_open_fraction_is_binomial(orc):
    seed, sweep = 99, 3
    thr = 2515933592
    n = 40000
    opened = sum(orc.bond_open(seed, sweep, thr, l, True) for l in range(n))
    p = thr / 2**32
    assert abs(opened - n * p) < 5 * math.sqrt(n * p * (1 - p))


def test_streams_are_keyed_by_seed_sweep_and_index(orc):
    a = [orc.flip_spin(5, 0, r) for r in range(256)]
    b = [orc.flip_spin(5, 1, r) for r in range(256)]
    c = [orc.flip_spin(6, 0, r) for r in range(256)]
    assert a != b and a != c
    ups = sum(1 for v in a if v > 0)
    assert 128 - 40 < ups < 128 + 40
    init = [orc.init_spin(1, i) for i in range(4096)]
    assert abs(sum(init)) < 5 * 64


# --------------------------------------------------------------------------- #
# Known answers for the initial-spin and cluster-flip layouts, rebuilt here
# from the Philox block alone (itself pinned above against ATen and rocRAND):
# the spin of index k is bit k mod 32 of word (k >> 5) mod 4 of the block
# k >> 7, counter (k >> 7, 0, sweep, tag), tag 0 for the start, 3 for flips.
# A wrong word index, bit index, block counter, sweep slot or tag in either
# oracle function changes some of these values.
# --------------------------------------------------------------------------- #
def _layout_bit(orc, seed, sweep, tag, k):
    blk = orc.philox([k >> 7, 0, sweep, tag], [seed & 0xFFFFFFFF, seed >> 32])
    return +1 if (int(blk[(k >> 5) & 3]) >> (k & 31)) & 1 else -1


def _layout_indices():
    rng = np.random.default_rng(41)
    # three whole blocks (every bit of every word), block and word edges, and
    # random indices up to the largest site index a lattice can have
    idx = list(range(0, 384)) + [127, 128, 129, 255, 256, 4095, 4096, 2**20 - 1, 2**20, 2**31 - 2]
    return idx + rng.integers(0, 2**31 - 1, size=500).tolist()


@pytest.mark.parametrize("seed", [1, 0xDEADBEEF12345678])
def test_initial_spin_layout_known_answers(orc, seed):
    for k in _layout_indices():
        assert orc.init_spin(seed, k) == _layout_bit(orc, seed, 0, 0, k), k


@pytest.mark.parametrize("seed,sweep", [(1, 0), (5, 1), (0xDEADBEEF12345678, 977)])
def test_flip_spin_layout_known_answers(orc, seed, sweep):
    for r in _layout_indices():
        assert orc.flip_spin(seed, sweep, r) == _layout_bit(orc, seed, sweep, 3, r), r


def test_initial_block_carries_all_128_bits(orc):
    """Sites 128..255 take the 128 bits of block 1 in order: word 0 bits 0..31,
    then word 1, 2, 3."""
    seed = 77
    blk = orc.philox([1, 0, 0, 0], [seed, 0])
    bits = [(int(blk[w]) >> b) & 1 for w in range(4) for b in range(32)]
    got = [1 if orc.init_spin(seed, 128 + j) > 0 else 0 for j in range(128)]
    assert got == bits


def test_lattice_start_and_flip_follow_the_layout(orc):
    """The lattice-level helpers use the same layout: the start of a 3D lattice
    and the flip of a labelled lattice, site by site."""
    dim, L, seed = 3, 9, 12345
    sp = orc.init_spins(dim, L, seed)
    assert [int(v) for v in sp] == [_layout_bit(orc, seed, 0, 0, k) for k in range(L ** dim)]
    rng = np.random.default_rng(5)
    labels = np.sort(rng.integers(0, L ** dim, size=L ** dim)).astype(np.int32)
    fl = orc.flip(dim, L, seed, 6, labels)
    assert [int(v) for v in fl] == [_layout_bit(orc, seed, 6, 3, int(r)) for r in labels]
