"""Batched mode and PCC feedback against the oracle (GPU).

Replicas of different dim, L, T, seeds and flags share every phase launch
(the sweeps of a call replayed from one hipGraph); each must follow exactly
the trajectory the oracle computes for it alone.  PCC replicas must reproduce the oracle's
percolation flags and p values bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu

MIX = [
    dict(dim=2, L=64, T=2.1, seed=11),
    dict(dim=2, L=100, T=workloads.TC_2D, seed=12),
    dict(dim=2, L=37, T=2.6, seed=13),
    dict(dim=3, L=16, T=workloads.TC_3D, seed=14),
    dict(dim=3, L=21, T=5.0, seed=15),
    dict(dim=2, L=130, T=2.4, seed=16),
]
PCC_MIX = [
    dict(dim=2, L=32, seed=21, p_bond=0.5, pcc=True, dp0=0.02, halve_every=7),
    dict(dim=3, L=12, seed=22, p_bond=0.3, pcc=True, dp0=0.01, halve_every=5),
    dict(dim=2, L=40, seed=23, p_bond=0.7, pcc=True),
]


def _params(spec, series=True, keep=True):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), series=series, keep_labels=keep, **s)


def _oracle(spec, nsweeps):
    if spec.get("pcc"):
        return oracle.run(spec["dim"], spec["L"], spec["seed"], nsweeps, p=spec["p_bond"], pcc=True,
                          dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000))
    return oracle.run(spec["dim"], spec["L"], spec["seed"], nsweeps, T=spec["T"])


def _check(lat, r, spec, ref):
    assert np.array_equal(lat.spins(r), ref["spins"]), f"spins of replica {r} {spec}"
    assert np.array_equal(lat.labels(r), ref["labels"]), f"labels of replica {r} {spec}"
    assert np.array_equal(lat.series(r), ref["series"]), f"series of replica {r} {spec}"
    if spec.get("pcc"):
        perc, p = lat.pcc_trace(r)
        assert np.array_equal(perc, ref["perc"]), f"percolation flags of replica {r}"
        assert np.array_equal(p, ref["p_trace"]), f"p trace of replica {r}"
        s, pp, thr = lat.state(r)
        assert pp == ref["p"] and thr == ref["thr"]


@pytest.mark.parametrize("calls", [(6,), (1, 4, 3), (2, 2, 2, 2)])
def test_batched_mix_matches_oracle(calls):
    specs = MIX + PCC_MIX
    total = sum(calls)
    with swgpu.Lattice([_params(s) for s in specs]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        for n in calls:
            lat.sweep(n)
        for r, spec in enumerate(specs):
            assert lat.state(r)[0] == total
            _check(lat, r, spec, _oracle(spec, total))


def test_batched_then_plain_then_batched():
    specs = MIX[:3] + PCC_MIX[:1]
    with swgpu.Lattice([_params(s) for s in specs]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(3)
        lat.set_mode(swgpu.SW_MODE_PLAIN)
        lat.sweep(2)
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(4)
        for r, spec in enumerate(specs):
            _check(lat, r, spec, _oracle(spec, 9))


def test_batched_tile_shapes_and_grid_do_not_change_results():
    specs = MIX
    ref = [_oracle(s, 3) for s in specs]
    for shape in range(len(swgpu.tile_shapes(2))):
        with swgpu.Lattice([_params(s) for s in specs]) as lat:
            for r in range(len(specs)):
                lat.set_tile_shape(r, shape)
            lat.set_mode(swgpu.SW_MODE_BATCHED)
            lat.sweep(3)
            for r, spec in enumerate(specs):
                _check(lat, r, spec, ref[r])


def test_autotune_keeps_trajectories(tmp_path):
    specs = MIX[:4]
    cache = str(tmp_path / "tune.json")
    with swgpu.Lattice([_params(s) for s in specs]) as lat:
        lat.autotune(sweeps=1, cache=cache)
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(3)
        for r, spec in enumerate(specs):
            _check(lat, r, spec, _oracle(spec, 3))
    import json

    entries = json.load(open(cache))
    assert entries and all(e["merge"] in (0, 64, 256) and e["engine"] in (0, 1) for e in entries.values())


def test_pcc_plain_matches_oracle_over_halvings():
    spec = dict(dim=2, L=48, seed=5, p_bond=0.5, pcc=True, dp0=0.01, halve_every=10)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.sweep(25)
        lat.sweep(15)
        _check(lat, 0, spec, _oracle(spec, 40))


def test_pcc_plain_trace_growth_keeps_device_p():
    """Growing the series and PCC traces between sweep calls rewrites the replica's
    descriptor; p and the bond threshold, which the feedback changed on the device,
    must survive that rewrite."""
    spec = dict(dim=2, L=40, seed=12, p_bond=0.5, pcc=True, dp0=0.02, halve_every=3, series_cap=4)
    with swgpu.Lattice(_params(spec)) as lat:
        for n in (3, 5, 9, 1):
            lat.sweep(n)
        _check(lat, 0, spec, _oracle(spec, 18))


@pytest.mark.parametrize("dim,L", [(2, 30), (3, 10)])
def test_pcc_rows_not_in_quads(dim, L):
    """PCC on lattices whose rows are not whole quads of sites (the flip kernel's
    per-site coverage marks), plain and batched."""
    spec = dict(dim=dim, L=L, seed=31, p_bond=0.45 if dim == 2 else 0.3, pcc=True, dp0=0.02, halve_every=5)
    ref = _oracle(spec, 12)
    for mode in (swgpu.SW_MODE_PLAIN, swgpu.SW_MODE_BATCHED):
        with swgpu.Lattice(_params(spec)) as lat:
            lat.set_mode(mode)
            lat.sweep(5)
            lat.sweep(7)
            _check(lat, 0, spec, ref)


def test_pcc_resume_sets_p():
    spec = dict(dim=2, L=24, seed=8, p_bond=0.5, pcc=True, dp0=0.02, halve_every=6)
    ref = _oracle(spec, 10)
    head = _oracle(spec, 6)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.set_spins(0, head["spins"], sweep=6, p=head["p"])
        lat.sweep(4)
        assert np.array_equal(lat.spins(), ref["spins"])
        assert lat.state()[1] == ref["p"]


def test_batched_workload_sample_replicas():
    """The 512-replica workload: a sample of replicas checked after 3 batched sweeps."""
    wl = workloads.batched()
    params = [swgpu.params_from_replica(r) for r in wl.replicas]
    sample = [0, 1, 2, 100, 257, 511]
    with swgpu.Lattice(params) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(3)
        for r in sample:
            rep = wl.replicas[r]
            ref = oracle.run(rep.dim, rep.L, rep.seed, 3, T=rep.T, keep_labels=False, record_series=False)
            assert np.array_equal(lat.spins(r), ref["spins"]), f"replica {r} (L={rep.L})"
