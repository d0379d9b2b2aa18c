"""Bit-packed spins (SW_BITPACK: one bit per site on the device) against the
oracle (GPU; through the C ABI).  Every result must be the one the int8 path
and the oracle give, bit for bit: rows that are whole bytes of bits (the flip
kernel's byte stores) and rows that are not (words shared between tiles,
updated by atomic AND / OR), 2D and 3D, with labels and series, PCC, the
batched engine with packed and int8 replicas mixed, the server, a bound
device tensor, and the plain workload's lattices at full size."""
import numpy as np
import pytest
import torch

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu

TC = workloads.TC_2D


def _params(spec, series=True, keep=True, bitpack=True):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), series=series, keep_labels=keep, bitpack=bitpack, **s)


def _oracle(spec, n, spins=None, s0=0):
    if spec.get("pcc"):
        return oracle.run(spec["dim"], spec["L"], spec["seed"], n, p=spec["p_bond"], pcc=True,
                          dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000), spins=spins, s0=s0)
    return oracle.run(spec["dim"], spec["L"], spec["seed"], n, T=spec["T"], spins=spins, s0=s0)


@pytest.mark.parametrize("dim,L,T", [(2, 64, TC), (2, 96, 2.4), (2, 100, TC), (2, 37, 2.1), (2, 130, 2.6),
                                     (3, 16, workloads.TC_3D), (3, 24, 5.0), (3, 13, 4.0)])
@pytest.mark.parametrize("keep", [False, True])
def test_plain_packed_matches_oracle(dim, L, T, keep):
    spec = dict(dim=dim, L=L, T=T, seed=300 + L)
    with swgpu.Lattice(_params(spec, keep=keep)) as lat:
        assert np.array_equal(lat.spins(), oracle.init_spins(dim, L, spec["seed"]))
        spins = oracle.init_spins(dim, L, spec["seed"])
        thr = lat.state()[2]
        for k in range(3):
            lat.sweep(1)
            spins, lab = oracle.sweep(dim, L, spec["seed"], k, thr, spins)
            assert np.array_equal(lat.spins(), spins), f"spins after sweep {k} ({dim}D L={L} keep={keep})"
            if keep:
                assert np.array_equal(lat.labels(), lab), f"labels after sweep {k}"
        assert np.array_equal(lat.series(), _oracle(spec, 3)["series"])
        assert lat.measure() == oracle.measure(dim, L, spins)


@pytest.mark.parametrize("dim,L", [(2, 70), (3, 19)])
def test_set_and_get_spins_roundtrip(dim, L):
    spec = dict(dim=dim, L=L, T=2.3 if dim == 2 else 4.6, seed=5)
    start = workloads.random_spins(dim, L, 77)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.set_spins(0, start, sweep=9)
        assert np.array_equal(lat.spins(), start)
        lat.sweep(2)
        ref = _oracle(spec, 2, spins=start, s0=9)
        assert np.array_equal(lat.spins(), ref["spins"])
        assert np.array_equal(lat.labels(), ref["labels"])


MIX = [
    (dict(dim=2, L=64, T=2.1, seed=11), True),
    (dict(dim=2, L=100, T=TC, seed=12), False),
    (dict(dim=2, L=37, T=2.6, seed=13), True),
    (dict(dim=3, L=16, T=workloads.TC_3D, seed=14), True),
    (dict(dim=3, L=21, T=5.0, seed=15), False),
    (dict(dim=2, L=130, T=2.4, seed=16), True),
    (dict(dim=2, L=48, seed=21, p_bond=0.55, pcc=True, dp0=0.02, halve_every=3), True),
    (dict(dim=3, L=12, seed=22, p_bond=0.3, pcc=True, dp0=0.01, halve_every=5), True),
]


@pytest.mark.parametrize("per_cu", [0, 2])
def test_batched_packed_and_int8_mixed(per_cu):
    with swgpu.Lattice([_params(s, bitpack=b) for s, b in MIX]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.set_batch_grid(per_cu)
        lat.sweep(2)
        lat.sweep(3)
        for r, (spec, b) in enumerate(MIX):
            ref = _oracle(spec, 5)
            assert np.array_equal(lat.spins(r), ref["spins"]), f"replica {r} {spec} packed={b}"
            assert np.array_equal(lat.labels(r), ref["labels"]), f"replica {r}"
            assert np.array_equal(lat.series(r), ref["series"]), f"replica {r}"
            if spec.get("pcc"):
                perc, pv = lat.pcc_trace(r)
                assert np.array_equal(perc, ref["perc"]) and np.array_equal(pv, ref["p_trace"]), f"replica {r}"


def test_bind_packed_device_tensor():
    """A bit-packed replica bound to a caller's int32 tensor of ceil(N/32) words."""
    dim, L, seed = 2, 96, 41
    spec = dict(dim=dim, L=L, T=2.5, seed=seed)
    start = workloads.random_spins(dim, L, 4)
    bits = np.zeros((L * L + 31) // 32, dtype=np.uint32)
    for i, v in enumerate(start):
        if v > 0:
            bits[i >> 5] |= np.uint32(1 << (i & 31))
    t = torch.from_numpy(bits.view(np.int32).copy()).to("cuda")
    ref = _oracle(spec, 4, spins=start)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.bind_device_spins(0, t)
        lat.sweep(4)
        assert np.array_equal(lat.spins(), ref["spins"])
        torch.cuda.synchronize()
    words = t.cpu().numpy().view(np.uint32)
    got = np.array([1 if (words[i >> 5] >> (i & 31)) & 1 else -1 for i in range(L * L)], dtype=np.int8)
    assert np.array_equal(got, ref["spins"])


def test_server_packed_jobs_equal_alone():
    jobs = [(dict(dim=2, L=40, T=2.2, seed=1), 9, True), (dict(dim=3, L=10, T=4.5, seed=2), 7, True),
            (dict(dim=2, L=77, T=TC, seed=3), 11, False), (dict(dim=2, L=64, T=2.0, seed=6), 5, True)]
    with swgpu.Server(hbm_budget=1 << 30, max_slots=3, sweeps_per_tick=4) as srv:
        ids = [srv.submit(_params(s, series=False, keep=False, bitpack=b), n) for s, n, b in jobs]
        for _ in range(1000):
            if srv.step() == 0:
                break
        for jid, (spec, n, b) in zip(ids, jobs):
            ref = _oracle(spec, n)["spins"]
            assert srv.poll(jid) == "done"
            assert np.array_equal(srv.spins(jid, spec["L"] ** spec["dim"]), ref), f"job {jid} packed={b}"
            assert srv.result(jid)["hash"] == swgpu.fnv1a64(ref)


def test_packed_footprint_is_smaller():
    a = swgpu.Server.footprint(swgpu.make_params(2, 4096))
    b = swgpu.Server.footprint(swgpu.make_params(2, 4096, bitpack=True))
    assert a - b == 4096 * 4096 - 4096 * 4096 // 8


@pytest.mark.parametrize("dim,L,T", [(2, 8192, TC), (3, 256, workloads.TC_3D)])
def test_full_size_packed(dim, L, T):
    """The plain workload's lattices bit-packed: two sweeps, every site compared."""
    spec = dict(dim=dim, L=L, T=T, seed=1)
    with swgpu.Lattice(_params(spec, series=False, keep=False)) as lat:
        thr = lat.state()[2]
        spins = oracle.init_spins(dim, L, 1)
        assert np.array_equal(lat.spins(), spins)
        for k in range(2):
            lat.sweep(1)
            spins, _ = oracle.sweep(dim, L, 1, k, thr, spins)
            assert np.array_equal(lat.spins(), spins), f"sweep {k}"
