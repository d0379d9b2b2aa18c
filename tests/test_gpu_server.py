"""Continuous-batching server (GPU): every job's result equals the same job
run alone, admission respects the memory budget and the slot count, and
cancellation frees resources.  Tolerance 0: results are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_0808_2109_amd import swgpu, workloads

pytestmark = pytest.mark.gpu

JOBS = [
    (dict(dim=2, L=40, T=2.2, seed=1), 17),
    (dict(dim=3, L=10, T=4.5, seed=2), 9),
    (dict(dim=2, L=77, T=workloads.TC_2D, seed=3), 31),
    (dict(dim=2, L=20, T=3.0, seed=4), 4),
    (dict(dim=3, L=17, T=4.0, seed=5), 22),
    (dict(dim=2, L=64, T=2.0, seed=6), 13),
    (dict(dim=2, L=33, seed=7, p_bond=0.5, pcc=True, dp0=0.02, halve_every=5), 12),
    (dict(dim=2, L=129, T=2.3, seed=8), 8),
    (dict(dim=3, L=8, T=6.0, seed=9), 1),
    (dict(dim=2, L=50, T=2.5, seed=10), 0),
]


def _params(spec):
    s = dict(spec)
    return swgpu.make_params(s.pop("dim"), s.pop("L"), **s)


def _alone(spec, n):
    if spec.get("pcc"):
        ref = oracle.run(spec["dim"], spec["L"], spec["seed"], n, p=spec["p_bond"], pcc=True,
                         dp0=spec.get("dp0", 0.01), halve_every=spec.get("halve_every", 1000))
    else:
        ref = oracle.run(spec["dim"], spec["L"], spec["seed"], n, T=spec["T"])
    return ref["spins"]


def _drain(srv, limit=10000):
    for _ in range(limit):
        if srv.step() == 0:
            return
    raise AssertionError("server did not drain")


def test_results_equal_alone_runs_in_the_mix():
    with swgpu.Server(hbm_budget=1 << 30, max_slots=4, sweeps_per_tick=5) as srv:
        ids = [srv.submit(_params(s), n) for s, n in JOBS[:5]]
        srv.step()                       # first jobs are running when the rest arrive
        ids += [srv.submit(_params(s), n) for s, n in JOBS[5:]]
        _drain(srv)
        for jid, (spec, n) in zip(ids, JOBS):
            assert srv.poll(jid) == "done"
            res = srv.result(jid)
            ref = _alone(spec, n)
            L, dim = spec["L"], spec["dim"]
            got = srv.spins(jid, L ** dim)
            assert np.array_equal(got, ref), f"job {jid} {spec}"
            assert res["hash"] == swgpu.fnv1a64(ref)
            assert (res["e_int"], res["m"]) == oracle.measure(dim, L, ref)
            assert res["t_submit"] <= res["t_start"] <= res["t_done"]
        st = srv.stats()
        assert st["done"] == len(JOBS) and st["bytes_in_use"] == 0


def test_admission_by_budget_and_rejection():
    big = _params(dict(dim=2, L=300, T=2.3, seed=1))
    small = _params(dict(dim=2, L=30, T=2.3, seed=2))
    fp_small = swgpu.Server.footprint(small)
    assert swgpu.Server.footprint(big) > 4 * fp_small
    # room for two small jobs at a time, never for the big one
    with swgpu.Server(hbm_budget=2 * fp_small + 10, max_slots=8, sweeps_per_tick=3) as srv:
        jb = srv.submit(big, 5)
        assert srv.poll(jb) == "rejected"
        ids = [srv.submit(_params(dict(dim=2, L=30, T=2.3, seed=s)), 7) for s in range(2, 7)]
        srv.step()
        running = [j for j in ids if srv.poll(j) == "running"]
        assert len(running) == 2
        assert srv.stats()["bytes_in_use"] <= 2 * fp_small + 10
        _drain(srv)
        for s, j in zip(range(2, 7), ids):
            ref = _alone(dict(dim=2, L=30, T=2.3, seed=s), 7)
            assert np.array_equal(srv.spins(j, 900), ref)
        assert srv.stats()["rejected"] == 1


def test_zero_budget_rejects_everything():
    with swgpu.Server(hbm_budget=0, max_slots=2, sweeps_per_tick=2) as srv:
        j = srv.submit(_params(dict(dim=2, L=16, T=2.0, seed=1)), 3)
        assert srv.poll(j) == "rejected"
        assert srv.step() == 0


def test_cancel_queued_and_running():
    with swgpu.Server(hbm_budget=1 << 30, max_slots=1, sweeps_per_tick=2) as srv:
        a = srv.submit(_params(dict(dim=2, L=40, T=2.2, seed=1)), 50)
        b = srv.submit(_params(dict(dim=2, L=40, T=2.2, seed=2)), 6)
        c = srv.submit(_params(dict(dim=2, L=40, T=2.2, seed=3)), 6)
        srv.step()
        assert srv.poll(a) == "running" and srv.poll(b) == "queued"
        srv.cancel(b)
        srv.cancel(a)
        assert srv.poll(a) == "cancelled" and srv.poll(b) == "cancelled"
        assert srv.stats()["bytes_in_use"] == 0
        _drain(srv)
        assert srv.poll(c) == "done"
        assert np.array_equal(srv.spins(c, 1600), _alone(dict(dim=2, L=40, T=2.2, seed=3), 6))
        with pytest.raises(swgpu.SwError):
            srv.result(a)
        with pytest.raises(swgpu.SwError):
            srv.poll(12345)
