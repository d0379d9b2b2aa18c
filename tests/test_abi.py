"""The C-ABI library loads and exports every entry point that include/sw_api.h
declares; parameter validation runs before any device call (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sw_api.h")
LIB = os.path.join(ROOT, "paper_0808_2109_amd", "libswgpu.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(sw_[a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_0808_2109_amd import build

        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sw_init", "sw_sweep", "sw_measure", "sw_get_series", "sw_get_spins", "sw_get_labels",
                 "sw_get_state", "sw_set_spins", "sw_free", "sw_last_error", "sw_server_create",
                 "sw_server_submit", "sw_server_step", "sw_server_result", "sw_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # nothing but the C ABI is exported
    assert all(n.startswith("sw_") for n in exported), sorted(n for n in exported if not n.startswith("sw_"))


def test_binding_loads_and_validates_without_device(lib_path):
    from paper_0808_2109_amd import swgpu

    lib = swgpu.lib()
    assert lib.sw_last_error()
    bad = [
        dict(dim=4, L=10), dict(dim=2, L=2), dict(dim=2, L=46341), dict(dim=3, L=1128),
        dict(dim=2, L=16, T=-1.0), dict(dim=2, L=16, J=-1.0), dict(dim=2, L=16, p_bond=1.5),
        dict(dim=2, L=16, pcc=True, dp0=0.0), dict(dim=2, L=16, pcc=True, halve_every=0),
    ]
    for kw in bad:
        p = swgpu.make_params(**kw)
        with pytest.raises(swgpu.SwError) as ei:
            swgpu.Lattice(p, stream=None)
        assert ei.value.code == swgpu.SW_EINVAL, kw
    # footprint is a pure host computation
    p = swgpu.make_params(2, 8192)
    fp = swgpu.Server.footprint(p)
    # spins 1 B, tile labels 2 B, border-merge slots, bitmaps and face ranks
    # under 1 B per site; kept labels add 8 B per site (labels and the border
    # roots' cluster roots)
    assert 3 * 8192 * 8192 <= fp < 4 * 8192 * 8192
    assert swgpu.Server.footprint(swgpu.make_params(2, 8192, keep_labels=True)) == fp + 8 * 8192 * 8192
    with pytest.raises(swgpu.SwError):
        swgpu.Server.footprint(swgpu.make_params(5, 8))


def test_tile_shapes_table(lib_path):
    from paper_0808_2109_amd import swgpu

    for dim in (2, 3):
        shapes = swgpu.tile_shapes(dim)
        assert len(shapes) >= 2
        for tx, ty, tz in shapes:
            assert tx % 16 == 0 and tx * ty * tz <= 32768 and ty * tz == 64
            assert (tz == 1) == (dim == 2)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark has a one-GPU path only: --gpus 2 stops with a message."""
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
