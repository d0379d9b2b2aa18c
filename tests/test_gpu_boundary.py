"""Boundary calls that earlier tests left out (GPU; through the C ABI).

* sw_set_spins on a handle that already ran past the resume point: the
  continuation must equal the oracle's run from the checkpoint, series rows and
  PCC traces included (rows restart at the resume point; no mark of the
  abandoned trajectory may survive).
* sw_bind_device_spins with a torch tensor as the lattice.
* The batched launch shape (sw_set_batch_grid): results may not depend on it.
* The border merge's schedule (sw_set_merge_width): neither may it.
* The persistent batched engine (sw_set_batch_engine): one cooperative launch
  with grid barriers must give what the phase kernels give.
* PCC across tiles in 2D, and at the PCC workload's lattice size (2048^2).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu

TC = workloads.TC_2D


def _params(spec, series=True, keep=True):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), series=series, keep_labels=keep, **s)


def _oracle(spec, nsweeps, s0=0, spins=None, p=None):
    if spec.get("pcc"):
        return oracle.run(spec["dim"], spec["L"], spec["seed"], nsweeps, p=spec["p_bond"] if p is None else p,
                          pcc=True, dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000),
                          s0=s0, spins=spins)
    return oracle.run(spec["dim"], spec["L"], spec["seed"], nsweeps, T=spec["T"], s0=s0, spins=spins)


REWIND = [
    dict(dim=2, L=70, T=2.3, seed=41),
    dict(dim=3, L=14, T=workloads.TC_3D, seed=42),
    dict(dim=2, L=48, seed=43, p_bond=0.62, pcc=True, dp0=0.004, halve_every=3),
    dict(dim=2, L=130, seed=44, p_bond=0.6, pcc=True, dp0=0.003, halve_every=4),
    dict(dim=3, L=12, seed=45, p_bond=0.35, pcc=True, dp0=0.003, halve_every=4),
]


@pytest.mark.parametrize("mode", [swgpu.SW_MODE_PLAIN, swgpu.SW_MODE_BATCHED])
def test_rewind_on_the_same_handle(mode):
    """Sweep 7, resume from the checkpoint of sweep 4 on the same handle, sweep
    3 more: spins, labels, the series rows of sweeps 4..6, the percolation flags
    and the p values must be those of the straight run."""
    full = [_oracle(s, 7) for s in REWIND]
    head = [_oracle(s, 4) for s in REWIND]
    with swgpu.Lattice([_params(s) for s in REWIND]) as lat:
        lat.set_mode(mode)
        lat.sweep(7)
        for r, spec in enumerate(REWIND):
            lat.set_spins(r, head[r]["spins"], sweep=4, p=head[r]["p"] if spec.get("pcc") else -1.0)
        lat.sweep(3)
        for r, spec in enumerate(REWIND):
            ref = full[r]
            assert np.array_equal(lat.spins(r), ref["spins"]), f"spins of replica {r} {spec}"
            assert np.array_equal(lat.labels(r), ref["labels"]), f"labels of replica {r} {spec}"
            rows, first = lat.series(r, with_first=True)
            assert first == 4
            assert np.array_equal(rows, ref["series"][4:7]), f"series of replica {r} {spec}"
            if spec.get("pcc"):
                perc, pv, tfirst = lat.pcc_trace(r, with_first=True)
                assert tfirst == 4
                assert np.array_equal(perc, ref["perc"][4:7]), f"percolation flags of replica {r}"
                assert np.array_equal(pv, ref["p_trace"][4:7]), f"p trace of replica {r}"
                s, p, thr = lat.state(r)
                assert (s, p, thr) == (7, ref["p"], ref["thr"])
        assert any(full[r]["perc"][4:7].any() for r in range(len(REWIND)) if REWIND[r].get("pcc")), \
            "the PCC cases should percolate in some compared sweep"


def test_resume_far_ahead_keeps_the_series_in_bounds():
    """A resume point beyond the series buffer: rows start there, and reading
    them never goes past the buffer."""
    spec = dict(dim=2, L=40, T=2.2, seed=7)
    start = workloads.random_spins(2, 40, 3)
    ref = _oracle(spec, 2, s0=5000, spins=start)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.sweep(2)
        lat.set_spins(0, start, sweep=5000)
        rows, first = lat.series(with_first=True)
        assert first == 5000 and rows.shape == (0, 2)
        lat.sweep(2)
        rows, first = lat.series(with_first=True)
        assert first == 5000
        assert np.array_equal(rows, ref["series"])
        assert np.array_equal(lat.spins(), ref["spins"])


@pytest.mark.parametrize("mode", [swgpu.SW_MODE_PLAIN, swgpu.SW_MODE_BATCHED])
def test_bind_device_spins_uses_the_torch_tensor(mode):
    """A caller-owned torch int8 tensor becomes the lattice: its contents are the
    start, the sweeps write into it, and the handle never frees it."""
    dim, L, seed = 2, 90, 17
    start = workloads.random_spins(dim, L, 99)
    spec = dict(dim=dim, L=L, T=2.4, seed=seed)
    ref = _oracle(spec, 5, spins=start)
    other = dict(dim=3, L=11, T=5.0, seed=18)
    ref_other = _oracle(other, 5)
    t = torch.from_numpy(start.copy()).to("cuda")
    with swgpu.Lattice([_params(spec), _params(other)]) as lat:
        lat.set_mode(mode)
        lat.bind_device_spins(0, t)
        lat.sweep(2)
        lat.sweep(3)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), ref["spins"])
        assert np.array_equal(lat.spins(0), ref["spins"])
        assert np.array_equal(lat.labels(0), ref["labels"])
        assert np.array_equal(lat.series(0), ref["series"])
        assert np.array_equal(lat.spins(1), ref_other["spins"])
    # still a valid tensor after the handle is gone
    assert int(t.abs().sum().item()) == L * L


def test_bind_device_spins_refuses_a_misaligned_tensor():
    L = 40
    base = torch.ones(L * L + 16, dtype=torch.int8, device="cuda")
    with swgpu.Lattice(swgpu.make_params(2, L, T=2.3, seed=3)) as lat:
        with pytest.raises(swgpu.SwError) as ei:
            lat.bind_device_spins(0, base[1:1 + L * L])       # 1 byte past a 16-byte boundary
        assert ei.value.code == swgpu.SW_EINVAL
        lat.bind_device_spins(0, base[16:16 + L * L])         # aligned: accepted


MIX = [
    dict(dim=2, L=64, T=2.1, seed=11),
    dict(dim=2, L=100, T=TC, seed=12),
    dict(dim=2, L=37, T=2.6, seed=13),
    dict(dim=3, L=16, T=workloads.TC_3D, seed=14),
    dict(dim=3, L=21, T=5.0, seed=15),
    dict(dim=2, L=130, T=2.4, seed=16),
    dict(dim=2, L=257, T=TC, seed=17),
    dict(dim=2, L=32, seed=21, p_bond=0.5, pcc=True, dp0=0.02, halve_every=7),
    dict(dim=3, L=12, seed=22, p_bond=0.3, pcc=True, dp0=0.01, halve_every=5),
    dict(dim=2, L=150, seed=23, p_bond=0.58, pcc=True, dp0=0.005, halve_every=2),
    dict(dim=2, L=1024, T=TC, seed=18),
]


@pytest.mark.parametrize("per_cu", [0, 1, 2, 4, 16])
def test_batched_grid_does_not_change_results(per_cu):
    """Every replica of the mix is checked against the oracle whatever the
    batched launch shape: one workgroup per tile, or 1 / 2 / 4 / 16 per CU (the
    mix has more tiles than 256 or 512 workgroups, so there each workgroup
    takes several tiles in turn)."""
    refs = [_oracle(s, 5) for s in MIX]
    for shape in range(len(swgpu.tile_shapes(2))):
        with swgpu.Lattice([_params(s) for s in MIX]) as lat:
            for r in range(len(MIX)):
                lat.set_tile_shape(r, shape)
            lat.set_mode(swgpu.SW_MODE_BATCHED)
            lat.set_batch_grid(per_cu)
            assert lat.batch_grid() == per_cu
            lat.sweep(2)
            lat.sweep(3)
            for r, spec in enumerate(MIX):
                ref = refs[r]
                assert np.array_equal(lat.spins(r), ref["spins"]), f"per_cu {per_cu} shape {shape} replica {r}"
                assert np.array_equal(lat.labels(r), ref["labels"]), f"per_cu {per_cu} shape {shape} replica {r}"
                assert np.array_equal(lat.series(r), ref["series"]), f"per_cu {per_cu} shape {shape} replica {r}"
                if spec.get("pcc"):
                    perc, pv = lat.pcc_trace(r)
                    assert np.array_equal(perc, ref["perc"]) and np.array_equal(pv, ref["p_trace"])


def test_batch_grid_rejects_out_of_range():
    with swgpu.Lattice(_params(dict(dim=2, L=16, T=2.0, seed=1))) as lat:
        for bad in (-1, 65):
            with pytest.raises(swgpu.SwError) as ei:
                lat.set_batch_grid(bad)
            assert ei.value.code == swgpu.SW_EINVAL


@pytest.mark.parametrize("mode", [swgpu.SW_MODE_PLAIN, swgpu.SW_MODE_BATCHED])
@pytest.mark.parametrize("width", [64, 256])
def test_merge_width_does_not_change_results(mode, width):
    """The border merge run with one wave or with 256 threads per tile, in
    every tile shape, plain and batched: every replica of the mix (2D and 3D,
    PCC among them) still matches the oracle."""
    refs = [_oracle(s, 5) for s in MIX]
    for shape in range(len(swgpu.tile_shapes(2))):
        with swgpu.Lattice([_params(s) for s in MIX]) as lat:
            for r in range(len(MIX)):
                lat.set_tile_shape(r, shape)
            lat.set_mode(mode)
            lat.set_merge_width(width)
            assert lat.merge_width() == width
            lat.sweep(2)
            lat.sweep(3)
            for r, spec in enumerate(MIX):
                ref = refs[r]
                tag = f"width {width} mode {mode} shape {shape} replica {r}"
                assert np.array_equal(lat.spins(r), ref["spins"]), tag
                assert np.array_equal(lat.labels(r), ref["labels"]), tag
                assert np.array_equal(lat.series(r), ref["series"]), tag
                if spec.get("pcc"):
                    perc, pv = lat.pcc_trace(r)
                    assert np.array_equal(perc, ref["perc"]) and np.array_equal(pv, ref["p_trace"]), tag


@pytest.mark.parametrize("per_cu", [0, 1])
def test_persistent_engine_matches_oracle(per_cu):
    """Every replica of the mix (2D and 3D, ragged, PCC among them) through the
    persistent engine, in both tile-shape pairs, with as many workgroups as fit
    and with one per CU (each then walks a long chunk of the list), over two
    calls; then the engine is switched back mid-run."""
    refs = [_oracle(s, 7) for s in MIX]
    for shape in range(len(swgpu.tile_shapes(2))):
        with swgpu.Lattice([_params(s) for s in MIX]) as lat:
            for r in range(len(MIX)):
                lat.set_tile_shape(r, shape)
            lat.set_mode(swgpu.SW_MODE_BATCHED)
            lat.set_batch_engine(swgpu.SW_ENGINE_PERSISTENT)
            lat.set_batch_grid(per_cu)
            lat.sweep(2)
            lat.sweep(3)
            engine, grid = lat.batch_engine()
            assert engine == swgpu.SW_ENGINE_PERSISTENT and grid >= 1
            if per_cu:
                assert grid <= 256 * per_cu
            lat.set_batch_engine(swgpu.SW_ENGINE_GRAPH)
            lat.sweep(2)
            for r, spec in enumerate(MIX):
                ref = refs[r]
                tag = f"per_cu {per_cu} shape {shape} replica {r}"
                assert np.array_equal(lat.spins(r), ref["spins"]), tag
                assert np.array_equal(lat.labels(r), ref["labels"]), tag
                assert np.array_equal(lat.series(r), ref["series"]), tag
                if spec.get("pcc"):
                    perc, pv = lat.pcc_trace(r)
                    assert np.array_equal(perc, ref["perc"]) and np.array_equal(pv, ref["p_trace"]), tag


def test_persistent_engine_long_call():
    """More sweeps in one call than one persistent launch runs (4096): the call
    is split into launches, with the series carried across them."""
    specs = [dict(dim=2, L=20, T=2.3, seed=61), dict(dim=3, L=6, T=4.0, seed=62)]
    with swgpu.Lattice([_params(s) for s in specs]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.set_batch_engine(swgpu.SW_ENGINE_PERSISTENT)
        lat.sweep(4100)
        for r, spec in enumerate(specs):
            ref = _oracle(spec, 4100)
            assert np.array_equal(lat.spins(r), ref["spins"])
            assert np.array_equal(lat.series(r), ref["series"])


def test_batch_engine_rejects_unknown():
    with swgpu.Lattice(_params(dict(dim=2, L=16, T=2.0, seed=1))) as lat:
        for bad in (-1, 2):
            with pytest.raises(swgpu.SwError) as ei:
                lat.set_batch_engine(bad)
            assert ei.value.code == swgpu.SW_EINVAL
        assert lat.batch_engine() == (swgpu.SW_ENGINE_GRAPH, 0)


def test_merge_width_rejects_other_values():
    with swgpu.Lattice(_params(dict(dim=2, L=16, T=2.0, seed=1))) as lat:
        for bad in (-1, 32, 128, 512):
            with pytest.raises(swgpu.SwError) as ei:
                lat.set_merge_width(bad)
            assert ei.value.code == swgpu.SW_EINVAL
        assert lat.merge_width() == 0


@pytest.mark.parametrize("L,shape", [(130, 0), (130, 1), (200, 1)])
def test_pcc_2d_across_tiles_plain(L, shape):
    """2D PCC on lattices of several tiles (ragged in both axes): candidate
    selection through border roots, several slots per tile, multi-word
    coverage bitmaps."""
    spec = dict(dim=2, L=L, seed=61 + L, p_bond=0.6, pcc=True, dp0=0.01, halve_every=4)
    ref = _oracle(spec, 14)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.set_tile_shape(0, shape)
        lat.sweep(6)
        lat.sweep(8)
        perc, pv = lat.pcc_trace()
        assert np.array_equal(perc, ref["perc"])
        assert np.array_equal(pv, ref["p_trace"])
        assert np.array_equal(lat.spins(), ref["spins"])
        assert np.array_equal(lat.labels(), ref["labels"])
        assert lat.state()[1:] == (ref["p"], ref["thr"])
    assert 0 < ref["perc"].sum() < len(ref["perc"])


def test_pcc_workload_size_batched():
    """The PCC workload's lattices (2D L=2048, p0=0.5, dp 0.01 halved every
    1000 sweeps) as the benchmark runs them, batched: three replicas over six
    sweeps, flags, p, spins and labels against the oracle."""
    wl = workloads.pcc(n=3, L=2048, sweeps=6)
    specs = [dict(dim=2, L=r.L, seed=r.seed, p_bond=r.p_bond, pcc=True, dp0=r.dp0, halve_every=r.halve_every)
             for r in wl.replicas]
    with swgpu.Lattice([_params(s, series=False) for s in specs]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(6)
        for r, spec in enumerate(specs):
            ref = _oracle(spec, 6)
            perc, pv = lat.pcc_trace(r)
            assert np.array_equal(perc, ref["perc"]), f"replica {r}"
            assert np.array_equal(pv, ref["p_trace"]), f"replica {r}"
            assert np.array_equal(lat.spins(r), ref["spins"]), f"replica {r}"
            assert np.array_equal(lat.labels(r), ref["labels"]), f"replica {r}"
