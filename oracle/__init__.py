"""CPU oracle for the Swendsen-Wang sweep (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
never calls the GPU library.

The arithmetic lives in ``sw_oracle.c`` (plain sequential C: one Philox call
per link, breadth-first clusters); this module compiles it with gcc and wraps
it with ctypes and numpy.  ``ranges.py`` holds the paper's interval form of the
projection operator used by the percolation test (Sec. III).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

INT8P = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
INT32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
INT64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
UINT8P = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
UINT32P = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` next to its source (plain gcc, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    c = ctypes
    lib.orc_philox4x32_10.argtypes = [UINT32P, UINT32P, UINT32P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_threshold_from_p.argtypes = [c.c_double]
    lib.orc_threshold_from_p.restype = c.c_uint64
    lib.orc_bond_probability.argtypes = [c.c_double, c.c_double]
    lib.orc_bond_probability.restype = c.c_double
    lib.orc_threshold.argtypes = [c.c_double, c.c_double]
    lib.orc_threshold.restype = c.c_uint64
    lib.orc_init_spin.argtypes = [c.c_uint64, c.c_uint32]
    lib.orc_init_spin.restype = c.c_int
    lib.orc_bond_open.argtypes = [c.c_uint64, c.c_uint32, c.c_uint64, c.c_uint32, c.c_int]
    lib.orc_bond_open.restype = c.c_int
    lib.orc_flip_spin.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32]
    lib.orc_flip_spin.restype = c.c_int
    lib.orc_validate.argtypes = [c.c_int, c.c_int]
    lib.orc_validate.restype = c.c_int
    lib.orc_init_spins.argtypes = [c.c_int, c.c_int, c.c_uint64, INT8P]
    lib.orc_init_spins.restype = None
    lib.orc_bonds.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_uint64, INT8P, UINT8P]
    lib.orc_bonds.restype = None
    lib.orc_label_bfs.argtypes = [c.c_int, c.c_int, UINT8P, INT32P]
    lib.orc_label_bfs.restype = c.c_int64
    lib.orc_flip.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, INT32P, INT8P]
    lib.orc_flip.restype = None
    lib.orc_measure.argtypes = [c.c_int, c.c_int, INT8P, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.orc_measure.restype = None
    lib.orc_sweep.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_uint64, INT8P, INT32P]
    lib.orc_sweep.restype = c.c_int
    lib.orc_percolates.argtypes = [c.c_int, c.c_int, INT32P]
    lib.orc_percolates.restype = c.c_int
    lib.orc_pcc_update.argtypes = [c.POINTER(c.c_double), c.POINTER(c.c_uint64), c.c_int,
                                   c.c_uint32, c.c_double, c.c_uint32]
    lib.orc_pcc_update.restype = None
    lib.orc_run.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_int32,
                            c.POINTER(c.c_uint64), c.POINTER(c.c_double), c.c_int, c.c_double,
                            c.c_uint32, INT8P, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.orc_run.restype = c.c_int
    lib.orc_bonds_open.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_uint64, INT8P, UINT8P]
    lib.orc_bonds_open.restype = None
    lib.orc_measure_open.argtypes = [c.c_int, c.c_int, INT8P, c.POINTER(c.c_int64), c.POINTER(c.c_int64)]
    lib.orc_measure_open.restype = None
    lib.orc_spans_open.argtypes = [c.c_int, c.c_int, INT32P]
    lib.orc_spans_open.restype = c.c_int
    lib.orc_winds.argtypes = [c.c_int, c.c_int, UINT8P]
    lib.orc_winds.restype = c.c_int
    lib.orc_run_bc.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_int32,
                               c.POINTER(c.c_uint64), c.POINTER(c.c_double), c.c_int, c.c_double,
                               c.c_uint32, INT8P, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.orc_run_bc.restype = c.c_int
    _lib = lib
    return lib


def nsites(dim: int, L: int) -> int:
    return L ** dim


# --------------------------------------------------------------------------- #
# Random stream (SWRNG-1) and threshold.
# --------------------------------------------------------------------------- #
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def bond_probability(J: float, T: float) -> float:
    return _load().orc_bond_probability(J, T)


def threshold(J: float, T: float) -> int:
    return int(_load().orc_threshold(J, T))


def threshold_from_p(p: float) -> int:
    return int(_load().orc_threshold_from_p(p))


def init_spin(seed: int, i: int) -> int:
    return _load().orc_init_spin(seed, i)


def bond_open(seed: int, sweep: int, thr: int, link: int, equal: bool) -> int:
    return _load().orc_bond_open(seed, sweep, thr, link, int(bool(equal)))


def flip_spin(seed: int, sweep: int, label: int) -> int:
    return _load().orc_flip_spin(seed, sweep, label)


# --------------------------------------------------------------------------- #
# Lattice-level steps.
# --------------------------------------------------------------------------- #
def validate(dim: int, L: int) -> bool:
    return _load().orc_validate(dim, L) == 0


def init_spins(dim: int, L: int, seed: int) -> np.ndarray:
    s = np.empty(nsites(dim, L), dtype=np.int8)
    _load().orc_init_spins(dim, L, seed, s)
    return s


def bonds(dim: int, L: int, seed: int, sweep: int, thr: int, spins: np.ndarray) -> np.ndarray:
    """Bond array, shape (dim, N): entry [d, i] is 1 when link (i, d) is open."""
    n = nsites(dim, L)
    out = np.zeros(dim * n, dtype=np.uint8)
    _load().orc_bonds(dim, L, seed, sweep, thr, np.ascontiguousarray(spins, dtype=np.int8), out)
    return out.reshape(dim, n)


def bonds_open(dim: int, L: int, seed: int, sweep: int, thr: int, spins: np.ndarray) -> np.ndarray:
    """Bond array with open boundaries: the links that would wrap are absent (0)."""
    n = nsites(dim, L)
    out = np.zeros(dim * n, dtype=np.uint8)
    _load().orc_bonds_open(dim, L, seed, sweep, thr, np.ascontiguousarray(spins, dtype=np.int8), out)
    return out.reshape(dim, n)


def measure_open(dim: int, L: int, spins: np.ndarray):
    e = ctypes.c_int64()
    m = ctypes.c_int64()
    _load().orc_measure_open(dim, L, np.ascontiguousarray(spins, dtype=np.int8), ctypes.byref(e), ctypes.byref(m))
    return int(e.value), int(m.value)


def spans_open(dim: int, L: int, labels: np.ndarray) -> bool:
    rc = _load().orc_spans_open(dim, L, np.ascontiguousarray(labels, dtype=np.int32))
    if rc < 0:
        raise MemoryError("oracle spanning test failed")
    return bool(rc)


def winds(dim: int, L: int, open_: np.ndarray) -> bool:
    rc = _load().orc_winds(dim, L, np.ascontiguousarray(open_.reshape(-1), dtype=np.uint8))
    if rc < 0:
        raise MemoryError("oracle winding test failed")
    return bool(rc)


def label_bfs(dim: int, L: int, open_: np.ndarray) -> np.ndarray:
    n = nsites(dim, L)
    lab = np.empty(n, dtype=np.int32)
    rc = _load().orc_label_bfs(dim, L, np.ascontiguousarray(open_.reshape(-1), dtype=np.uint8), lab)
    if rc < 0:
        raise MemoryError("oracle labelling failed")
    return lab


def flip(dim: int, L: int, seed: int, sweep: int, labels: np.ndarray) -> np.ndarray:
    s = np.empty(nsites(dim, L), dtype=np.int8)
    _load().orc_flip(dim, L, seed, sweep, np.ascontiguousarray(labels, dtype=np.int32), s)
    return s


def measure(dim: int, L: int, spins: np.ndarray):
    e = ctypes.c_int64()
    m = ctypes.c_int64()
    _load().orc_measure(dim, L, np.ascontiguousarray(spins, dtype=np.int8), ctypes.byref(e), ctypes.byref(m))
    return int(e.value), int(m.value)


def sweep(dim: int, L: int, seed: int, sweep_index: int, thr: int, spins: np.ndarray):
    """One sweep; returns (new spins, labels).  The input array is not modified."""
    s = np.array(spins, dtype=np.int8, copy=True)
    lab = np.empty(nsites(dim, L), dtype=np.int32)
    if _load().orc_sweep(dim, L, seed, sweep_index, thr, s, lab) != 0:
        raise MemoryError("oracle sweep failed")
    return s, lab


def percolates(dim: int, L: int, labels: np.ndarray) -> bool:
    rc = _load().orc_percolates(dim, L, np.ascontiguousarray(labels, dtype=np.int32))
    if rc < 0:
        raise MemoryError("oracle percolation test failed")
    return bool(rc)


def pcc_update(p: float, thr: int, percolating: bool, sweep_index: int,
               dp0: float = 0.01, halve_every: int = 1000):
    pp = ctypes.c_double(p)
    tt = ctypes.c_uint64(thr)
    _load().orc_pcc_update(ctypes.byref(pp), ctypes.byref(tt), int(bool(percolating)),
                           sweep_index, dp0, halve_every)
    return pp.value, int(tt.value)


def run(dim: int, L: int, seed: int, nsweeps: int, *, thr: int | None = None, J: float = 1.0,
        T: float | None = None, p: float | None = None, s0: int = 0, spins: np.ndarray | None = None,
        pcc: bool = False, dp0: float = 0.01, halve_every: int = 1000,
        record_series: bool = True, keep_labels: bool = True, open_bc: bool = False, wind: bool = False):
    """Run `nsweeps` sweeps from sweep index s0.

    Returns a dict with spins, series (nsweeps x 2 of E_int, M), labels of the
    last sweep, and for pcc the percolation flags, the p trace and final p/thr.
    open_bc: open boundaries (PCC spanning: both opposite boundaries of an axis);
    wind: the topological rule instead of the extension rule (periodic only).
    """
    n = nsites(dim, L)
    if spins is None:
        spins = init_spins(dim, L, seed)
    s = np.array(spins, dtype=np.int8, copy=True)
    if p is None:
        p = bond_probability(J, T) if T is not None else 0.5
    if thr is None:
        thr = threshold_from_p(p) if (pcc or T is None) else threshold(J, T)
    tt = ctypes.c_uint64(thr)
    pp = ctypes.c_double(p)
    series = np.zeros((nsweeps, 2), dtype=np.int64) if record_series else None
    labels = np.zeros(n, dtype=np.int32) if keep_labels else None
    perc = np.zeros(nsweeps, dtype=np.int32) if pcc else None
    ptr = np.zeros(nsweeps, dtype=np.float64) if pcc else None

    def ptr_of(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)

    mode = (1 if pcc else 0) | (2 if open_bc else 0) | (4 if wind else 0)
    rc = _load().orc_run_bc(dim, L, seed, s0, nsweeps, ctypes.byref(tt), ctypes.byref(pp), mode,
                            dp0, halve_every, s, ptr_of(series), ptr_of(labels), ptr_of(perc), ptr_of(ptr))
    if rc != 0:
        raise ValueError("oracle run failed (invalid parameters or out of memory)")
    return {"spins": s, "series": series, "labels": labels, "perc": perc, "p_trace": ptr,
            "p": pp.value, "thr": int(tt.value)}
