"""ctypes binding of libswgpu.so (argument marshalling only).

Every step of a sweep runs in the HIP library; this module converts Python
values and numpy / torch buffers into the C ABI declared in include/sw_api.h
and raises SwError on a negative status.  There is no fallback: importing the
binding without a built library raises, and so does any call that needs a GPU
on a machine without one.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswgpu.so")

SW_OK, SW_EINVAL, SW_ENOMEM, SW_EHIP, SW_EBUSY, SW_ENOTFOUND, SW_ECANCELLED, SW_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
SW_RECORD_SERIES, SW_KEEP_LABELS, SW_PCC, SW_BITPACK, SW_OPEN, SW_PCC_WIND = 1, 2, 4, 8, 16, 32
SW_MODE_PLAIN, SW_MODE_BATCHED = 0, 1
SW_ENGINE_GRAPH, SW_ENGINE_PERSISTENT = 0, 1
JOB_STATES = {0: "queued", 1: "running", 2: "done", 3: "rejected", 4: "cancelled"}
PHASES = ("k1_bond_label", "k2_merge", "k3_flip", "pcc", "measure", "batched", "k3_resolve")


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class sw_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("J", ctypes.c_double),
        ("T", ctypes.c_double),
        ("p_bond", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("pcc_dp0", ctypes.c_double),
        ("pcc_halve_every", ctypes.c_uint32),
        ("series_cap", ctypes.c_uint32),
    ]


_lib = None


def _torch_first():
    # torch ships its own HIP runtime under the same soname; loading it first
    # makes the library and torch share one runtime (and one set of streams)
    try:
        import torch  # noqa: F401
    except Exception:  # pragma: no cover
        pass


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_0808_2109_amd.build")
    _torch_first()
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp = c.c_void_p
    P = c.POINTER
    sig = {
        "sw_params_default": (None, [P(sw_params)]),
        "sw_last_error": (c.c_char_p, []),
        "sw_init": (c.c_int, [P(sw_params), c.c_int32, c.c_int32, vp, P(vp)]),
        "sw_set_mode": (c.c_int, [vp, c.c_int32]),
        "sw_set_batch_grid": (c.c_int, [vp, c.c_int32]),
        "sw_get_batch_grid": (c.c_int, [vp, P(c.c_int32)]),
        "sw_set_merge_width": (c.c_int, [vp, c.c_int32]),
        "sw_set_batch_engine": (c.c_int, [vp, c.c_int32]),
        "sw_get_batch_engine": (c.c_int, [vp, P(c.c_int32), P(c.c_int32)]),
        "sw_get_merge_width": (c.c_int, [vp, P(c.c_int32)]),
        "sw_sweep": (c.c_int, [vp, c.c_int32]),
        "sw_sweep_replica": (c.c_int, [vp, c.c_int32, c.c_int32]),
        "sw_measure": (c.c_int, [vp, c.c_int32, P(c.c_int64), P(c.c_int64)]),
        "sw_get_series": (c.c_int, [vp, c.c_int32, vp, c.c_int64, P(c.c_int64), P(c.c_int64)]),
        "sw_get_spins": (c.c_int, [vp, c.c_int32, vp, c.c_int64]),
        "sw_get_labels": (c.c_int, [vp, c.c_int32, vp, c.c_int64]),
        "sw_get_state": (c.c_int, [vp, c.c_int32, P(c.c_uint32), P(c.c_double), P(c.c_uint64)]),
        "sw_get_pcc_trace": (c.c_int, [vp, c.c_int32, vp, vp, c.c_int64, P(c.c_int64), P(c.c_int64)]),
        "sw_set_spins": (c.c_int, [vp, c.c_int32, vp, c.c_int64, c.c_uint32, c.c_double]),
        "sw_bind_device_spins": (c.c_int, [vp, c.c_int32, vp]),
        "sw_set_timing": (c.c_int, [vp, c.c_int32]),
        "sw_get_timing": (c.c_int, [vp, P(c.c_double), P(c.c_int64), c.c_int32]),
        "sw_set_tile_shape": (c.c_int, [vp, c.c_int32, c.c_int32]),
        "sw_get_tile_shape": (c.c_int, [vp, c.c_int32, P(c.c_int32)]),
        "sw_tile_shapes": (c.c_int, [c.c_int32, P(c.c_int32), P(c.c_int32), P(c.c_int32), P(c.c_int32), c.c_int32]),
        "sw_autotune": (c.c_int, [vp, c.c_int32, c.c_char_p]),
        "sw_free": (c.c_int, [vp]),
        "sw_sweep_noalloc": (c.c_int, [P(sw_params), vp, c.c_uint32, c.c_int32, vp, vp, vp, vp]),
        "sw_server_create": (c.c_int, [c.c_uint64, c.c_int32, c.c_int32, c.c_int32, vp, P(vp)]),
        "sw_server_submit": (c.c_int, [vp, P(sw_params), c.c_int32, P(c.c_uint64)]),
        "sw_server_footprint": (c.c_int, [P(sw_params), P(c.c_uint64)]),
        "sw_server_poll": (c.c_int, [vp, c.c_uint64, P(c.c_int32)]),
        "sw_server_result": (c.c_int, [vp, c.c_uint64, P(c.c_int64), P(c.c_int64), P(c.c_uint64),
                                       P(c.c_double), P(c.c_double), P(c.c_double)]),
        "sw_server_spins": (c.c_int, [vp, c.c_uint64, vp, c.c_int64]),
        "sw_server_cancel": (c.c_int, [vp, c.c_uint64]),
        "sw_server_step": (c.c_int, [vp, P(c.c_int32)]),
        "sw_server_stats": (c.c_int, [vp, P(c.c_int64), P(c.c_int64), P(c.c_double), P(c.c_uint64)]),
        "sw_server_now": (c.c_int, [vp, P(c.c_double)]),
        "sw_server_destroy": (c.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            raise RuntimeError(f"{LIB_PATH} does not export {name}; rebuild it")
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != SW_OK:
        raise SwError(rc, lib().sw_last_error().decode())


def default_stream():
    """torch's current stream as a hipStream_t handle, or None without a GPU."""
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover
        pass
    return None


def make_params(dim: int = 2, L: int = 64, T: Optional[float] = None, seed: int = 1, J: float = 1.0,
                p_bond: float = -1.0, series: bool = False, keep_labels: bool = False, pcc: bool = False,
                dp0: float = 0.01, halve_every: int = 1000, series_cap: int = 0, bitpack: bool = False,
                open_bc: bool = False, wind: bool = False) -> sw_params:
    p = sw_params()
    lib().sw_params_default(ctypes.byref(p))
    p.dim, p.L, p.J, p.seed = dim, L, J, seed
    if T is not None:
        p.T = T
    p.p_bond = p_bond
    p.flags = ((SW_RECORD_SERIES if series else 0) | (SW_KEEP_LABELS if keep_labels else 0) | (SW_PCC if pcc else 0)
               | (SW_BITPACK if bitpack else 0) | (SW_OPEN if open_bc else 0) | (SW_PCC_WIND if wind else 0))
    p.pcc_dp0, p.pcc_halve_every, p.series_cap = dp0, halve_every, series_cap
    return p


def params_from_replica(rep, series=False, keep_labels=False) -> sw_params:
    """Build sw_params from a workloads.Replica."""
    return make_params(rep.dim, rep.L, rep.T, rep.seed, rep.J, rep.p_bond, series=series,
                       keep_labels=keep_labels, pcc=rep.pcc, dp0=rep.dp0, halve_every=rep.halve_every)


def tile_shapes(dim: int):
    n = ctypes.c_int32()
    tx = (ctypes.c_int32 * 16)()
    ty = (ctypes.c_int32 * 16)()
    tz = (ctypes.c_int32 * 16)()
    _check(lib().sw_tile_shapes(dim, ctypes.byref(n), tx, ty, tz, 16))
    return [(tx[i], ty[i], tz[i]) for i in range(n.value)]


class Lattice:
    """A handle holding one or more replicas (sw_init ... sw_free)."""

    def __init__(self, params: Sequence[sw_params] | sw_params, device: int = -1, stream="torch"):
        if isinstance(params, sw_params):
            params = [params]
        self.params: List[sw_params] = list(params)
        arr = (sw_params * len(self.params))(*self.params)
        if stream == "torch":
            stream = default_stream()
        self._h = ctypes.c_void_p()
        _check(lib().sw_init(arr, len(self.params), device, stream, ctypes.byref(self._h)))

    # -- lifecycle
    def close(self):
        if self._h:
            lib().sw_free(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nsites(self, r: int = 0) -> int:
        return self.params[r].L ** self.params[r].dim

    # -- sweeps
    def set_mode(self, mode: int):
        _check(lib().sw_set_mode(self._h, mode))

    def set_batch_grid(self, per_cu: int):
        """Workgroups per CU of batched sweeps (0: one per tile)."""
        _check(lib().sw_set_batch_grid(self._h, per_cu))

    def batch_grid(self) -> int:
        v = ctypes.c_int32()
        _check(lib().sw_get_batch_grid(self._h, ctypes.byref(v)))
        return int(v.value)

    def set_batch_engine(self, engine: int):
        """SW_ENGINE_GRAPH (phase kernels in a replayed graph) or SW_ENGINE_PERSISTENT."""
        _check(lib().sw_set_batch_engine(self._h, engine))

    def batch_engine(self):
        """(engine, workgroups of the last persistent launch)."""
        e, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sw_get_batch_engine(self._h, ctypes.byref(e), ctypes.byref(g)))
        return int(e.value), int(g.value)

    def set_merge_width(self, threads: int):
        """Threads per tile of the border merge (0: per tile shape, 64 or 256)."""
        _check(lib().sw_set_merge_width(self._h, threads))

    def merge_width(self) -> int:
        v = ctypes.c_int32()
        _check(lib().sw_get_merge_width(self._h, ctypes.byref(v)))
        return int(v.value)

    def sweep(self, n: int = 1):
        _check(lib().sw_sweep(self._h, n))

    def sweep_replica(self, r: int, n: int = 1):
        _check(lib().sw_sweep_replica(self._h, r, n))

    # -- read back
    def measure(self, r: int = 0):
        e = ctypes.c_int64()
        m = ctypes.c_int64()
        _check(lib().sw_measure(self._h, r, ctypes.byref(e), ctypes.byref(m)))
        return int(e.value), int(m.value)

    def series(self, r: int = 0, with_first: bool = False):
        """(E_int, M) rows of the sweeps first, first + 1, ... (first = the last resume point)."""
        st = self.state(r)
        cap = 2 * max(st[0], 1)
        buf = np.zeros(cap, dtype=np.int64)
        cnt = ctypes.c_int64()
        first = ctypes.c_int64()
        _check(lib().sw_get_series(self._h, r, buf.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(cnt),
                                   ctypes.byref(first)))
        rows = buf[: 2 * cnt.value].reshape(-1, 2)
        return (rows, int(first.value)) if with_first else rows

    def spins(self, r: int = 0) -> np.ndarray:
        n = self.nsites(r)
        buf = np.empty(n, dtype=np.int8)
        _check(lib().sw_get_spins(self._h, r, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def labels(self, r: int = 0) -> np.ndarray:
        n = self.nsites(r)
        buf = np.empty(n, dtype=np.int32)
        _check(lib().sw_get_labels(self._h, r, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def state(self, r: int = 0):
        s = ctypes.c_uint32()
        p = ctypes.c_double()
        t = ctypes.c_uint64()
        _check(lib().sw_get_state(self._h, r, ctypes.byref(s), ctypes.byref(p), ctypes.byref(t)))
        return int(s.value), float(p.value), int(t.value)

    def pcc_trace(self, r: int = 0, with_first: bool = False):
        """Percolation flags and p after each feedback step, from sweep `first` on."""
        n = self.state(r)[0]
        perc = np.zeros(max(n, 1), dtype=np.int32)
        pv = np.zeros(max(n, 1), dtype=np.float64)
        cnt = ctypes.c_int64()
        first = ctypes.c_int64()
        _check(lib().sw_get_pcc_trace(self._h, r, perc.ctypes.data_as(ctypes.c_void_p),
                                      pv.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(cnt), ctypes.byref(first)))
        out = (perc[: cnt.value], pv[: cnt.value])
        return (*out, int(first.value)) if with_first else out

    # -- write
    def set_spins(self, r: int, spins: np.ndarray, sweep: int = 0, p: float = -1.0):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        _check(lib().sw_set_spins(self._h, r, s.ctypes.data_as(ctypes.c_void_p), s.size, sweep, p))

    def bind_device_spins(self, r: int, tensor):
        """Use a caller-owned torch CUDA tensor as the spin array: int8 of N
        elements, or for a bit-packed replica int32 of ceil(N/32) words."""
        if self.params[r].flags & SW_BITPACK:
            ok = str(tensor.dtype) == "torch.int32" and tensor.numel() == (self.nsites(r) + 31) // 32
        else:
            ok = str(tensor.dtype) == "torch.int8" and tensor.numel() == self.nsites(r)
        if not ok or not tensor.is_contiguous() or not tensor.is_cuda:
            raise ValueError("need a contiguous device tensor: int8 of N, or int32 of ceil(N/32) when bit-packed")
        self._bound = getattr(self, "_bound", {})
        self._bound[r] = tensor                   # keep it alive while bound
        _check(lib().sw_bind_device_spins(self._h, r, ctypes.c_void_p(tensor.data_ptr())))

    # -- tuning / timing
    def set_tile_shape(self, r: int, shape: int):
        _check(lib().sw_set_tile_shape(self._h, r, shape))

    def tile_shape(self, r: int = 0) -> int:
        s = ctypes.c_int32()
        _check(lib().sw_get_tile_shape(self._h, r, ctypes.byref(s)))
        return int(s.value)

    def autotune(self, sweeps: int = 3, cache: Optional[str] = None):
        _check(lib().sw_autotune(self._h, sweeps, cache.encode() if cache else None))

    def set_timing(self, on: bool = True):
        _check(lib().sw_set_timing(self._h, 1 if on else 0))

    def timing(self):
        k = len(PHASES)
        ms = (ctypes.c_double * k)()
        n = (ctypes.c_int64 * k)()
        _check(lib().sw_get_timing(self._h, ms, n, k))
        return {PHASES[i]: (float(ms[i]), int(n[i])) for i in range(k)}


def sweep_noalloc(params: sw_params, spins, n_sweeps: int, sweep0: int = 0, series=None, labels=None, err=None,
                  stream="torch"):
    """sw_sweep_noalloc on caller-owned torch device tensors (spins int8 of N;
    optional series int64 of 2*n_sweeps, labels int32 of N, err int32 of 1)."""
    def ptr(t, dtype, n):
        if t is None:
            return None
        if str(t.dtype) != dtype or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"need a contiguous {dtype} device tensor of {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    n = params.L ** params.dim
    if stream == "torch":
        stream = default_stream()
    _check(lib().sw_sweep_noalloc(ctypes.byref(params), ptr(spins, "torch.int8", n), sweep0, n_sweeps,
                                  ptr(series, "torch.int64", 2 * n_sweeps), ptr(labels, "torch.int32", n),
                                  ptr(err, "torch.int32", 1), stream))


class Server:
    """Continuous-batching job server (sw_server_*)."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, sweeps_per_tick: int = 10, device: int = -1,
                 stream="torch"):
        if stream == "torch":
            stream = default_stream()
        self._s = ctypes.c_void_p()
        _check(lib().sw_server_create(hbm_budget, max_slots, sweeps_per_tick, device, stream, ctypes.byref(self._s)))

    def close(self):
        if self._s:
            lib().sw_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def footprint(p: sw_params) -> int:
        b = ctypes.c_uint64()
        _check(lib().sw_server_footprint(ctypes.byref(p), ctypes.byref(b)))
        return int(b.value)

    def submit(self, p: sw_params, n_sweeps: int) -> int:
        j = ctypes.c_uint64()
        _check(lib().sw_server_submit(self._s, ctypes.byref(p), n_sweeps, ctypes.byref(j)))
        return int(j.value)

    def poll(self, job: int) -> str:
        st = ctypes.c_int32()
        _check(lib().sw_server_poll(self._s, job, ctypes.byref(st)))
        return JOB_STATES[st.value]

    def result(self, job: int) -> dict:
        e = ctypes.c_int64()
        m = ctypes.c_int64()
        h = ctypes.c_uint64()
        t0 = ctypes.c_double()
        t1 = ctypes.c_double()
        t2 = ctypes.c_double()
        _check(lib().sw_server_result(self._s, job, ctypes.byref(e), ctypes.byref(m), ctypes.byref(h),
                                      ctypes.byref(t0), ctypes.byref(t1), ctypes.byref(t2)))
        return {"e_int": e.value, "m": m.value, "hash": h.value, "t_submit": t0.value, "t_start": t1.value,
                "t_done": t2.value}

    def spins(self, job: int, n: int) -> np.ndarray:
        buf = np.empty(n, dtype=np.int8)
        _check(lib().sw_server_spins(self._s, job, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def cancel(self, job: int):
        _check(lib().sw_server_cancel(self._s, job))

    def step(self) -> int:
        a = ctypes.c_int32()
        _check(lib().sw_server_step(self._s, ctypes.byref(a)))
        return int(a.value)

    def stats(self) -> dict:
        d = ctypes.c_int64()
        r = ctypes.c_int64()
        su = ctypes.c_double()
        b = ctypes.c_uint64()
        _check(lib().sw_server_stats(self._s, ctypes.byref(d), ctypes.byref(r), ctypes.byref(su), ctypes.byref(b)))
        return {"done": d.value, "rejected": r.value, "site_updates": su.value, "bytes_in_use": b.value}

    def now(self) -> float:
        t = ctypes.c_double()
        _check(lib().sw_server_now(self._s, ctypes.byref(t)))
        return t.value


def fnv1a64(spins: np.ndarray) -> int:
    """64-bit FNV-1a of a spin array's bytes (the hash sw_server_result reports)."""
    h = 0xCBF29CE484222325
    for b in np.ascontiguousarray(spins, dtype=np.int8).view(np.uint8).tobytes():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h
