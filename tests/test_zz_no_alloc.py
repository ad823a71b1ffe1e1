"""lbm3_mass_device, the entry point that allocates nothing: its masses equal lbm3_mass's bit for
bit, through the C ABI, on two calls in a row (the second on a smaller context, so the fixed
scratch array of the library is reused with fewer chunks)."""
import numpy as np
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


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_mass_device_equals_mass(precision):
    torch, lbm3 = _mods()
    big = [W.random_mixture(200, 96, seed=5, walls=True, circles=[(60.3, 40.2, 11.0), (140.7, 55.1, 9.0)]),
           W.pillar_domain(2102_007)]
    small = [W.random_mixture(40, 20, seed=6, walls=True)]
    for case, ws in (("big", big), ("small", small)):
        print(f"no-alloc: {case} context, {len(ws)} domain(s), {precision}", flush=True)
        sim = lbm3.Simulation(ws, precision=precision)
        sim.step(7)
        ref = sim.mass()
        out = sim.mass_device()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), (case, got, ref)
        assert np.all(np.isfinite(got)) and np.all(got > 0)
        sim.close()


def test_mass_device_rejects_contexts_beyond_its_scratch():
    """A context with 65537 chunks of 16 rows (one 3 x 1 048 577 periodic column of one fluid) is
    refused with LBM3_EINVAL before any launch; lbm3_mass still serves it.  A null output is
    refused too."""
    torch, lbm3 = _mods()
    ny = 16 * 65536 + 1
    rho = np.zeros((3, ny, 3))
    rho[2] = 1.0
    w = W.Workload("tall", 3, ny, 1, W.BC_PERIODIC, (0.1,) * 3, (0.01,) * 3, (90.0, 90.0),
                   np.zeros((ny, 3), np.uint8), rho)
    print("no-alloc: 3 x 1048577 column, f32 (over the scratch limit)", flush=True)
    sim = lbm3.Simulation([w], precision="f32")
    out = torch.zeros((1, 3), dtype=torch.float64, device=sim.device)
    with pytest.raises(lbm3.Lbm3Error) as e:
        sim.mass_device(out)
    assert e.value.code == lbm3.LBM3_EINVAL and "65536" in str(e.value)
    m = sim.mass()
    assert abs(m[0, 2] - 3 * ny) < 1e-6 * 3 * ny
    with pytest.raises(lbm3.Lbm3Error) as e:
        lbm3.lbm3_mass_device(sim.ctx, 0)
    assert e.value.code == lbm3.LBM3_EINVAL
    sim.close()
