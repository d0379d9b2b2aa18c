"""Open boundaries (SW_OPEN) against the oracle (GPU; through the C ABI).

The links that would wrap around the box do not exist: spins, labels and the
(E_int, M) series must equal the oracle's open-box run bit for bit, on
lattices of one tile and of many (ragged) tiles, 2D and 3D, int8 and
bit-packed, plain and batched with periodic replicas mixed in, and through
the server.  PCC on an open box uses the spanning test (one cluster holds
sites of both opposite faces of an axis): flags and p must follow the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu

TC = workloads.TC_2D


def _params(spec, series=True, keep=True):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), series=series, keep_labels=keep, **s)


def _oracle(spec, n):
    open_bc = spec.get("open_bc", False)
    if spec.get("pcc"):
        return oracle.run(spec["dim"], spec["L"], spec["seed"], n, p=spec["p_bond"], pcc=True, open_bc=open_bc,
                          dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000))
    return oracle.run(spec["dim"], spec["L"], spec["seed"], n, T=spec["T"], open_bc=open_bc)


@pytest.mark.parametrize("dim,L,T", [(2, 37, 2.1), (2, 64, TC), (2, 100, TC), (2, 130, 2.0), (2, 257, TC),
                                     (3, 13, 4.0), (3, 16, workloads.TC_3D), (3, 33, 4.5)])
@pytest.mark.parametrize("bitpack", [False, True])
def test_open_sweeps_match_oracle(dim, L, T, bitpack):
    spec = dict(dim=dim, L=L, T=T, seed=500 + L, open_bc=True, bitpack=bitpack)
    ref = _oracle(spec, 4)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.sweep(1)
        lat.sweep(3)
        assert np.array_equal(lat.spins(), ref["spins"]), f"{dim}D L={L} packed={bitpack}"
        assert np.array_equal(lat.labels(), ref["labels"])
        assert np.array_equal(lat.series(), ref["series"])
        assert lat.measure() == oracle.measure_open(dim, L, ref["spins"])
    # the boundary matters: the periodic run differs
    assert not np.array_equal(oracle.run(dim, L, 500 + L, 4, T=T)["labels"], ref["labels"])


def test_open_every_tile_shape():
    for dim, L, T in ((2, 100, TC), (3, 27, workloads.TC_3D)):
        spec = dict(dim=dim, L=L, T=T, seed=77, open_bc=True)
        ref = _oracle(spec, 2)
        for shape in range(len(swgpu.tile_shapes(dim))):
            with swgpu.Lattice(_params(spec)) as lat:
                lat.set_tile_shape(0, shape)
                lat.sweep(2)
                assert np.array_equal(lat.labels(), ref["labels"]), (dim, shape)
                assert np.array_equal(lat.spins(), ref["spins"]), (dim, shape)


@pytest.mark.parametrize("dim,L,p,shape", [(2, 40, 0.55, 0), (2, 130, 0.58, 0), (2, 130, 0.58, 1), (3, 12, 0.3, 0),
                                           (3, 20, 0.32, 0)])
def test_open_pcc_spanning_matches_oracle(dim, L, p, shape):
    spec = dict(dim=dim, L=L, seed=60 + L, p_bond=p, pcc=True, open_bc=True, dp0=0.01, halve_every=4)
    ref = _oracle(spec, 14)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.set_tile_shape(0, shape)
        lat.sweep(5)
        lat.sweep(9)
        perc, pv = lat.pcc_trace()
        assert np.array_equal(perc, ref["perc"])
        assert np.array_equal(pv, ref["p_trace"])
        assert np.array_equal(lat.spins(), ref["spins"])
        assert np.array_equal(lat.labels(), ref["labels"])
    assert 0 < ref["perc"].sum() < len(ref["perc"])


MIX = [
    dict(dim=2, L=64, T=2.1, seed=11, open_bc=True),
    dict(dim=2, L=100, T=TC, seed=12),
    dict(dim=2, L=37, T=2.6, seed=13, open_bc=True, bitpack=True),
    dict(dim=3, L=16, T=workloads.TC_3D, seed=14, open_bc=True),
    dict(dim=3, L=21, T=5.0, seed=15),
    dict(dim=2, L=48, seed=21, p_bond=0.55, pcc=True, dp0=0.02, halve_every=3, open_bc=True),
    dict(dim=2, L=48, seed=21, p_bond=0.55, pcc=True, dp0=0.02, halve_every=3),
    dict(dim=3, L=12, seed=22, p_bond=0.3, pcc=True, dp0=0.01, halve_every=5, open_bc=True),
]


@pytest.mark.parametrize("engine", [swgpu.SW_ENGINE_GRAPH, swgpu.SW_ENGINE_PERSISTENT])
def test_open_and_periodic_batched_together(engine):
    """Open and periodic boxes, int8 and bit-packed, PCC among them, in one
    batch: through the phase-kernel graph and through the persistent kernel."""
    with swgpu.Lattice([_params(s) for s in MIX]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.set_batch_engine(engine)
        lat.sweep(3)
        lat.sweep(3)
        for r, spec in enumerate(MIX):
            ref = _oracle(spec, 6)
            assert np.array_equal(lat.spins(r), ref["spins"]), f"replica {r} {spec}"
            assert np.array_equal(lat.labels(r), ref["labels"]), f"replica {r}"
            assert np.array_equal(lat.series(r), ref["series"]), f"replica {r}"
            if spec.get("pcc"):
                perc, pv = lat.pcc_trace(r)
                assert np.array_equal(perc, ref["perc"]) and np.array_equal(pv, ref["p_trace"]), f"replica {r}"


def test_open_jobs_through_the_server():
    jobs = [(dict(dim=2, L=40, T=2.2, seed=1, open_bc=True), 9), (dict(dim=3, L=10, T=4.5, seed=2, open_bc=True), 7),
            (dict(dim=2, L=40, T=2.2, seed=1), 9)]
    with swgpu.Server(hbm_budget=1 << 30, max_slots=2, sweeps_per_tick=4) as srv:
        ids = [srv.submit(_params(s, series=False, keep=False), n) for s, n in jobs]
        for _ in range(1000):
            if srv.step() == 0:
                break
        for jid, (spec, n) in zip(ids, jobs):
            ref = _oracle(spec, n)["spins"]
            assert np.array_equal(srv.spins(jid, spec["L"] ** spec["dim"]), ref), f"job {jid}"
