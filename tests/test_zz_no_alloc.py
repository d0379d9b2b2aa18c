"""sw_sweep_noalloc (the sweep for callers that cannot allocate) against the
handle path it is a variant of: sw_init + sw_set_spins + sw_sweep, bit for bit,
on two calls in a row on the same device (the second on a smaller lattice, so
the shared static scratch array holds the first call's leftovers), plus its
refusals.  GPU; calls go through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu


def _handle_path(dim, L, T, seed, start, sweep0, n):
    prm = swgpu.make_params(dim, L, T=T, seed=seed, series=True, keep_labels=True)
    with swgpu.Lattice(prm) as lat:
        lat.set_spins(0, start, sweep=sweep0)
        lat.sweep(n)
        return lat.spins(), lat.labels(), lat.series()


def _noalloc(dim, L, T, seed, start, sweep0, n):
    prm = swgpu.make_params(dim, L, T=T, seed=seed)
    spins = torch.from_numpy(start.copy()).to("cuda")
    series = torch.full((2 * n,), 12345, dtype=torch.int64, device="cuda")   # the call clears it
    labels = torch.full((L ** dim,), -7, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    swgpu.sweep_noalloc(prm, spins, n, sweep0=sweep0, series=series, labels=labels, err=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    return spins.cpu().numpy(), labels.cpu().numpy(), series.cpu().numpy().reshape(-1, 2)


CALLS = [
    (2, 300, 2.3, 5, 3, 4),            # 5 x 5 tiles, ragged
    (2, 70, workloads.TC_2D, 6, 0, 3),  # smaller: the scratch array still holds the first call's data
    (3, 40, workloads.TC_3D, 7, 11, 3),
    (3, 17, 5.0, 8, 2, 2),
]


def test_noalloc_equals_the_handle_path_on_consecutive_calls():
    for dim, L, T, seed, sweep0, n in CALLS:
        start = workloads.random_spins(dim, L, 1000 + seed)
        got = _noalloc(dim, L, T, seed, start, sweep0, n)
        want = _handle_path(dim, L, T, seed, start, sweep0, n)
        for g, w, what in zip(got, want, ("spins", "labels", "series")):
            assert np.array_equal(g, w), f"{what} differ (dim={dim} L={L} sweep0={sweep0} n={n})"
        ref = oracle.run(dim, L, seed, n, T=T, s0=sweep0, spins=start)
        assert np.array_equal(got[0], ref["spins"]) and np.array_equal(got[1], ref["labels"])
        assert np.array_equal(got[2], ref["series"])


@pytest.mark.parametrize("dim,L,T", [(3, 128, workloads.TC_3D), (2, 1448, workloads.TC_2D)])
def test_noalloc_at_the_largest_size(dim, L, T):
    """The largest lattices the static scratch array takes (2^21 sites), with
    labels and series, then a small one on the leftovers: equal to the handle
    path bit for bit."""
    for d, l, t, seed, sweep0, n in ((dim, L, T, 21, 7, 2), (2, 50, 2.4, 22, 0, 2)):
        start = workloads.random_spins(d, l, 500 + seed)
        got = _noalloc(d, l, t, seed, start, sweep0, n)
        want = _handle_path(d, l, t, seed, start, sweep0, n)
        for g, w, what in zip(got, want, ("spins", "labels", "series")):
            assert np.array_equal(g, w), f"{what} differ (dim={d} L={l})"


def test_noalloc_without_optional_outputs():
    dim, L, T, seed = 2, 128, 2.2, 9
    start = workloads.random_spins(dim, L, 3)
    spins = torch.from_numpy(start.copy()).to("cuda")
    swgpu.sweep_noalloc(swgpu.make_params(dim, L, T=T, seed=seed), spins, 5, sweep0=1)
    torch.cuda.synchronize()
    ref = oracle.run(dim, L, seed, 5, T=T, s0=1, spins=start)
    assert np.array_equal(spins.cpu().numpy(), ref["spins"])


def test_noalloc_refuses_what_it_cannot_do():
    big = swgpu.make_params(2, 1449, T=2.3, seed=1)          # 1449^2 > 2^21 sites
    pcc = swgpu.make_params(2, 64, seed=1, p_bond=0.5, pcc=True)
    for prm in (big, pcc):
        # refused on the host, before anything is enqueued: the pointer is never used
        rc = swgpu.lib().sw_sweep_noalloc(prm, swgpu.ctypes.c_void_p(16), 0, 1, None, None, None, None)
        assert rc == swgpu.SW_EINVAL
    ok = swgpu.make_params(2, 64, T=2.3, seed=1)
    assert swgpu.lib().sw_sweep_noalloc(ok, None, 0, 1, None, None, None, None) == swgpu.SW_EINVAL
    # a spin array that is not 16-byte aligned is refused before it is touched
    assert swgpu.lib().sw_sweep_noalloc(ok, swgpu.ctypes.c_void_p(4097), 0, 1, None, None, None, None) == swgpu.SW_EINVAL
