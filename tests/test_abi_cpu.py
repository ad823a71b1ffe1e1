"""CPU checks of the C ABI: the library loads, exports every declared symbol, and validates its
inputs on the host (no device call is made by lbm3_workspace_bytes)."""
import os
import re

import numpy as np
import pytest

from paper_2102_04709_amd import lbm3, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2102_04709_amd import build
    build.build(force=False)
    return lbm3.library()


def test_header_symbols_exported(lib):
    text = open(os.path.join(ROOT, "include", "lbm3.h")).read()
    declared = set(re.findall(r"\b(lbm3_[a-z_]+)\s*\(", text))
    assert declared == set(lbm3.ABI_SYMBOLS), declared ^ set(lbm3.ABI_SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def _bytes(ws, **opt):
    return lbm3.lbm3_workspace_bytes(lbm3.DomainArgs(ws), lbm3.make_options(**opt))


def test_workspace_size_scales_with_precision(lib):
    w = W.flat_janus()
    b64, b32, b16 = (_bytes([w], precision=p) for p in ("f64", "f32", "f16"))
    assert b64 > b32 > b16 > 0
    # two state buffers dominate: 2 * (9 S + 3 T) per padded node
    pitch, rows = 128, w.ny + 4
    assert b32 >= 2 * pitch * rows * (9 * 4 + 3 * 4)
    assert _bytes([w, w], precision="f32") > 1.9 * b32


@pytest.mark.parametrize("mutate,msg", [
    (dict(sigma=(0.0, 0.01, 0.01)), "tension"),
    (dict(nu=(4.0, 0.1, 0.1)), "tau"),
    (dict(theta_deg=(40.0, 110.0)), "Eq. (18)"),
    (dict(theta_deg=(0.0, 90.0)), "contact angles"),
])
def test_invalid_parameters_rejected(lib, mutate, msg):
    w = W.flat_janus().with_params(**mutate)
    with pytest.raises(lbm3.Lbm3Error) as e:
        _bytes([w])
    assert e.value.code == lbm3.LBM3_EINVAL and msg in str(e.value)


def test_invalid_geometry_rejected(lib):
    # an isolated single solid node has no defined normal (Eq. 19 sums to zero)
    w = W.random_mixture(20, 20, seed=1, walls=False)
    s = w.solid.copy()
    s[10, 10] = 1
    with pytest.raises(lbm3.Lbm3Error, match="normal"):
        _bytes([w.with_params(solid=s)])
    # Zou-He needs periodic y and no solid next to the inlet
    w = W.pillar_domain(5, nx=120, ny=60, n_pillars=2)
    s = w.solid.copy()
    s[30, 1] = 1
    with pytest.raises(lbm3.Lbm3Error, match="Zou-He"):
        _bytes([w.with_params(solid=s)])
    with pytest.raises(lbm3.Lbm3Error):
        _bytes([w], tile=(8, 8))  # tile area below the minimum is an invalid option at create only


@pytest.mark.parametrize("precision,n", [("f64", 23200), ("f32", 32768), ("f16", 32768)])
def test_oversized_plane_rejected(lib, precision, n):
    """A domain plane whose byte offsets would not fit 32 bits is refused before any of its host
    arrays is read (the struct is given a small workload's arrays and an oversized shape)."""
    args = lbm3.DomainArgs([W.flat_janus()])
    args.array[0].nx = n
    args.array[0].ny = n
    with pytest.raises(lbm3.Lbm3Error, match="padded plane") as e:
        lbm3.lbm3_workspace_bytes(args, lbm3.make_options(precision=precision))
    assert e.value.code == lbm3.LBM3_EINVAL


def test_bad_options_rejected(lib):
    w = W.flat_janus()
    with pytest.raises(lbm3.Lbm3Error):
        _bytes([w], precision=7)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built HIP library the binding raises instead of computing."""
    monkeypatch.setattr(lbm3, "LIB_PATH", str(tmp_path / "liblbm3.so"))
    monkeypatch.setattr(lbm3, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        lbm3.library()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus 2 exits with status 2 and says so."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
