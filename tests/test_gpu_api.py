"""C-ABI behaviour on the GPU that is not arithmetic: the autotuner's JSON cache."""
import json

import pytest

from paper_2102_04709_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_04709_amd import lbm3
    lbm3.library()
    return torch, lbm3


def test_tune_cache_round_trip(tmp_path):
    """The first autotune times the candidates and stores its pick; a second context with the same
    shapes and precision takes the stored pick without running a step; another workload adds an
    entry."""
    torch, lbm3 = _mods()
    path = str(tmp_path / "tune.json")
    w = W.random_mixture(160, 96, seed=3, walls=True, circles=[(80.2, 47.9, 12.0)])
    print("tune cache: first autotune (timed)", flush=True)
    s1 = lbm3.Simulation(w, precision="f32", kernel="auto", tune_cache=path)
    c1 = s1.autotune(3)
    assert s1.query(7) > 0  # the candidates' warm-up steps advanced the state
    data = json.load(open(path))
    assert len(data) == 1
    (key, entry), = data.items()
    assert "f32" in key and "domains=1" in key
    assert (entry["kernel"], entry["tile_x"], entry["tile_y"]) == c1
    s1.close()
    print("tune cache: second autotune (cached)", flush=True)
    s2 = lbm3.Simulation(w, precision="f32", kernel="auto", tune_cache=path)
    c2 = s2.autotune(3)
    assert c2 == c1 and s2.query(7) == 0
    assert (s2.query(8), s2.query(4), s2.query(5)) == c1
    s2.close()
    s3 = lbm3.Simulation(W.random_mixture(96, 64, seed=4, walls=True), precision="f32", kernel="auto",
                         tune_cache=path)
    s3.autotune(2)
    s3.close()
    assert len(json.load(open(path))) == 2


def test_non_finite_density_is_reported():
    """Failure detection: a NaN planted in the state (at one fluid node's first partial density)
    makes lbm3_mass return LBM3_ENUMERIC, and the allocation-free mass shows a non-finite sum;
    stepping on goes on without a fault."""
    torch, lbm3 = _mods()
    w = W.random_mixture(48, 24, seed=8, walls=True)
    sim = lbm3.Simulation(w, precision="f32")
    sim.step(3)
    st = sim.get_state()
    f = st.view(torch.float32)
    pitch = (w.nx + 63) // 64 * 64
    plane = pitch * (w.ny + 4)
    j, i = 10, 20
    assert w.solid[j, i] == 0
    f[9 * plane + i + pitch * (j + 2)] = float("nan")
    sim.set_state(st)
    with pytest.raises(lbm3.Lbm3Error) as e:
        sim.mass()
    assert e.value.code == lbm3.LBM3_ENUMERIC
    sim.step(2)
    m = sim.mass_device()
    torch.cuda.synchronize()
    assert not bool(torch.isfinite(m).all())
    sim.close()


def test_library_loaded_before_torch():
    """A process that loads the library before anything imports torch still runs a step: the
    loader brings torch's HIP runtime up first, so the library shares it (with the system runtime
    loaded first, the runtime that comes with torch later finds no device)."""
    _mods()
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2102_04709_amd import lbm3, workloads as W\n"
            "assert 'torch' not in sys.modules\n"
            "lbm3.library()\n"
            "sim = lbm3.Simulation(W.random_mixture(64, 48, seed=1), precision='f32')\n"
            "sim.step(2)\n"
            "print('mass', float(sim.mass().sum()))\n" % root)
    print("library before torch: subprocess", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mass" in r.stdout
