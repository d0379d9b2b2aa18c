"""The topological (winding) percolation rule (SW_PCC | SW_PCC_WIND) against
the oracle (GPU; through the C ABI).

A cluster winds when it holds a loop around the periodic box.  The border
merge tracks each tile cluster's sheet of the unwrapped cover and flags a link
that closes a loop with a nonzero sheet shift; the flags, p, spins and labels
must follow the oracle's (a breadth-first search with unwrapped positions)
bit for bit, on one-tile lattices (every wrap a self-link of the tile), many
ragged tiles in both tile shapes, 3D, bit-packed, and in a batch with
extension-rule and open-box replicas.
"""
import numpy as np
import pytest

import oracle
from paper_0808_2109_amd import swgpu

pytestmark = pytest.mark.gpu


def _params(spec, series=True, keep=True):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), series=series, keep_labels=keep, **s)


def _oracle(spec, n):
    if spec.get("pcc"):
        return oracle.run(spec["dim"], spec["L"], spec["seed"], n, p=spec["p_bond"], pcc=True,
                          open_bc=spec.get("open_bc", False), wind=spec.get("wind", False),
                          dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000))
    return oracle.run(spec["dim"], spec["L"], spec["seed"], n, T=spec["T"])


@pytest.mark.parametrize("dim,L,p,shape,bitpack", [(2, 24, 0.6, 0, False), (2, 64, 0.6, 1, False),
                                                   (2, 130, 0.59, 0, False), (2, 130, 0.59, 1, True),
                                                   (2, 200, 0.59, 0, False), (3, 12, 0.3, 0, False),
                                                   (3, 20, 0.3, 1, True)])
def test_winding_rule_matches_oracle(dim, L, p, shape, bitpack):
    spec = dict(dim=dim, L=L, seed=90 + L, p_bond=p, pcc=True, wind=True, dp0=0.01, halve_every=4,
                bitpack=bitpack)
    ref = _oracle(spec, 14)
    with swgpu.Lattice(_params(spec)) as lat:
        lat.set_tile_shape(0, shape)
        lat.sweep(4)
        lat.sweep(10)
        perc, pv = lat.pcc_trace()
        assert np.array_equal(perc, ref["perc"]), (perc, ref["perc"])
        assert np.array_equal(pv, ref["p_trace"])
        assert np.array_equal(lat.spins(), ref["spins"])
        assert np.array_equal(lat.labels(), ref["labels"])
        assert np.array_equal(lat.series(), ref["series"])
    assert 0 < ref["perc"].sum() < len(ref["perc"])
    # the rule is not the extension rule: its trajectory differs
    ext = oracle.run(dim, L, 90 + L, 14, p=p, pcc=True, dp0=0.01, halve_every=4)
    assert not np.array_equal(ext["perc"], ref["perc"])


def test_winding_rule_rejects_open_boxes():
    for kw in (dict(wind=True), dict(pcc=True, wind=True, open_bc=True)):
        with pytest.raises(swgpu.SwError) as ei:
            swgpu.Lattice(swgpu.make_params(2, 32, p_bond=0.5, **kw))
        assert ei.value.code == swgpu.SW_EINVAL


MIX = [
    dict(dim=2, L=24, seed=31, p_bond=0.6, pcc=True, wind=True, dp0=0.01, halve_every=3),
    dict(dim=2, L=24, seed=31, p_bond=0.6, pcc=True, dp0=0.01, halve_every=3),
    dict(dim=2, L=24, seed=31, p_bond=0.6, pcc=True, open_bc=True, dp0=0.01, halve_every=3),
    dict(dim=2, L=100, seed=32, p_bond=0.59, pcc=True, wind=True, dp0=0.01, halve_every=3),
    dict(dim=3, L=12, seed=33, p_bond=0.3, pcc=True, wind=True, dp0=0.01, halve_every=3),
    dict(dim=2, L=70, T=2.3, seed=34),
]


@pytest.mark.parametrize("per_cu,engine", [(0, swgpu.SW_ENGINE_GRAPH), (1, swgpu.SW_ENGINE_GRAPH),
                                           (0, swgpu.SW_ENGINE_PERSISTENT)])
def test_winding_in_a_batch(per_cu, engine):
    with swgpu.Lattice([_params(s) for s in MIX]) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.set_batch_grid(per_cu)
        lat.set_batch_engine(engine)
        lat.sweep(5)
        lat.sweep(7)
        for r, spec in enumerate(MIX):
            ref = _oracle(spec, 12)
            assert np.array_equal(lat.spins(r), ref["spins"]), f"replica {r} {spec}"
            assert np.array_equal(lat.labels(r), ref["labels"]), f"replica {r}"
            if spec.get("pcc"):
                perc, pv = lat.pcc_trace(r)
                assert np.array_equal(perc, ref["perc"]), f"replica {r}: {perc} {ref['perc']}"
                assert np.array_equal(pv, ref["p_trace"]), f"replica {r}"
