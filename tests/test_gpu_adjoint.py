"""The hand-written adjoint of the step (lbm3_adjoint_*) and the differentiable rollout.

Gradients of a phase-field mismatch loss L = sum over fluid nodes of sum_k (C_k - C*_k)^2 at the
last step, with respect to (theta13, theta23, sigma12, sigma13, sigma23), are checked against
central finite differences of the FP64 oracle:
  - small domains covering every boundary rule (walls with the wetting fill, curved
    interpolated bounce-back, the fluid-exchanging periodic boundary, Zou-He inlet/outlet),
    FP64 adjoint, tight tolerance;
  - the 512 x 256 twelve-pillar inverse problem, 4000 steps with checkpoints every 100, FP32
    forward and adjoint, against oracle differences stored in tests/golden/adjoint_fd.json
    (written by tests/golden/make_adjoint_fd.py, which calls only the oracle), relative error
    1e-3.
The adjoint of the state is checked separately: <lambda_0, delta> against a central difference
of the loss along a random direction delta of the initial state.
"""
import json
import os

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_2102_04709_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_04709_amd import lbm3, rollout
    lbm3.library()
    return torch, lbm3, rollout


def mismatch(C, target, solid):
    """sum over fluid nodes and fluids of (C - target)^2, numpy FP64."""
    fl = solid == 0
    return float(((C - target)[:, fl] ** 2).sum())


def oracle_C(w, steps):
    o = po.Oracle(w)
    o.step(steps)
    r = o.rho()
    fl = w.solid == 0
    tot = np.where(fl, r.sum(0), 1.0)
    return np.where(fl, r / tot, 0.0)


def oracle_fd(w, steps, target, h):
    """Central differences of the oracle's loss in the five public parameters."""
    p0 = np.array([*w.theta_deg, *w.sigma], dtype=np.float64)
    g = np.zeros(5)
    for k in range(5):
        vals = []
        for sgn in (1, -1):
            p = p0.copy()
            p[k] += sgn * h[k]
            wk = w.with_params(theta_deg=(p[0], p[1]), sigma=(p[2], p[3], p[4]))
            vals.append(mismatch(oracle_C(wk, steps), target, w.solid))
        g[k] = (vals[0] - vals[1]) / (2 * h[k])
    return g


def gpu_grad(torch, lbm3, rollout, w, steps, target, precision, every):
    sim = lbm3.Simulation(w, precision=precision, adjoint=True)
    s0 = sim.get_state()
    params = rollout.params_of([w]).requires_grad_(True)
    rho = rollout.rollout(params, sim, steps, s0, every)
    C = rollout.phase_fields(rho, [w])[0]
    fl = torch.as_tensor(w.solid == 0, device=C.device)
    tgt = torch.as_tensor(target, device=C.device, dtype=C.dtype)
    L = (((C - tgt) ** 2) * fl).sum()
    L.backward()
    g = params.grad.numpy()[0].copy()
    sim.close()
    return float(L.detach().cpu()), g


def target_setup(w):
    """The same set-up at other parameters (a valid point of Eq. 18): the loss's target."""
    return w.with_params(theta_deg=(w.theta_deg[0] - 8.0, w.theta_deg[1] + 6.0),
                         sigma=tuple(s * f for s, f in zip(w.sigma, (1.1, 0.95, 1.05))))


def small_cases():
    return {
        "walls_circle": W.random_mixture(64, 40, 11, walls=True, circles=[(30.3, 19.6, 7.2)]),
        "periodic": W.random_mixture(40, 32, 12, walls=False),
        "swap13": W.random_mixture(48, 32, 13, walls=True, bc_x=W.BC_PERIODIC_SWAP13),
        "zouhe_circle": W.random_mixture(64, 32, 14, walls=False, y_periodic=1, bc_x=W.BC_ZOUHE,
                                         circles=[(31.5, 15.7, 6.4)]),
    }


# Steps per case: the discrete update is only piecewise smooth (the A_kl clamp of Eq. 10, the
# max/min of Eq. 22, the |G| threshold of the normals); with an inflow the fronts of the
# A_kl clamp sweep nodes quickly and kinks of L(p) come within the difference steps after
# ~25 steps, so that case runs fewer steps.
STEPS = {"walls_circle": 40, "periodic": 40, "swap13": 40, "zouhe_circle": 15}


@pytest.mark.parametrize("case", list(small_cases().keys()))
def test_adjoint_small_vs_oracle_fd(case):
    torch, lbm3, rollout = _mods()
    w = small_cases()[case]
    steps = STEPS[case]
    target = oracle_C(target_setup(w), steps)
    L, g = gpu_grad(torch, lbm3, rollout, w, steps, target, "f64", every=7)
    L_or = mismatch(oracle_C(w, steps), target, w.solid)
    h = np.array([1e-3, 1e-3, *(1e-5 * np.array(w.sigma))])
    g_fd = oracle_fd(w, steps, target, h)
    print(f"{case}: L gpu {L:.15e} oracle {L_or:.15e}", flush=True)
    print(f"{case}: adjoint {g}\n{case}: oracle fd {g_fd}", flush=True)
    assert abs(L - L_or) <= 1e-10 * max(1.0, abs(L_or))
    scale = np.abs(g_fd).max()
    assert scale > 0
    err = np.abs(g - g_fd) / np.maximum(np.abs(g_fd), 1e-3 * scale)
    print(f"{case}: rel err {err}", flush=True)
    assert err.max() <= 1e-5


def test_adjoint_batched_domains_vs_oracle_fd():
    """Two domains of different sizes and boundary rules advanced and differentiated together:
    each domain's gradient against the oracle's central differences of that domain alone."""
    torch, lbm3, rollout = _mods()
    cases = small_cases()
    ws = [cases["walls_circle"], cases["swap13"]]
    steps = 30
    targets = [oracle_C(target_setup(w), steps) for w in ws]
    sim = lbm3.Simulation(ws, precision="f64", adjoint=True)
    s0 = sim.get_state()
    params = rollout.params_of(ws).requires_grad_(True)
    rho = rollout.rollout(params, sim, steps, s0, 8)
    Cs = rollout.phase_fields(rho, ws)
    L = 0
    for C, w, t in zip(Cs, ws, targets):
        fl = torch.as_tensor(w.solid == 0, device=C.device)
        L = L + (((C - torch.as_tensor(t, device=C.device)) ** 2) * fl).sum()
    L.backward()
    g = params.grad.numpy()
    sim.close()
    for d, (w, t) in enumerate(zip(ws, targets)):
        h = np.array([1e-3, 1e-3, *(1e-5 * np.array(w.sigma))])
        g_fd = oracle_fd(w, steps, t, h)
        scale = np.abs(g_fd).max()
        err = np.abs(g[d] - g_fd) / np.maximum(np.abs(g_fd), 1e-3 * scale)
        print(f"domain {d}: adjoint {g[d]}\n  oracle fd {g_fd}\n  rel err {err}", flush=True)
        assert err.max() <= 1e-5


def _fluid_state_mask(w, precision_bytes=8, solid=False):
    """Mask of the state entries (12 planes: 9 distributions, 3 densities) at fluid nodes (at
    solid nodes with solid=True), in the state layout of a single domain: planes of
    pitch * (ny + 4) elements, pitch = nx rounded up to 64, node (i, j) at i + pitch * (j + 2)."""
    pitch = (w.nx + 63) // 64 * 64
    P = pitch * (w.ny + 4)
    m = np.zeros((12, P), bool)
    jj, ii = np.nonzero((w.solid != 0) if solid else (w.solid == 0))
    li = ii + pitch * (jj + 2)
    m[:, li] = True
    return m.reshape(-1)


def test_adjoint_of_state_directional():
    torch, lbm3, rollout = _mods()
    w = W.random_mixture(64, 40, 21, walls=True, circles=[(33.2, 20.4, 6.8)])
    steps = 10
    target = oracle_C(w.with_params(theta_deg=(55.0, 105.0)), steps)
    sim = lbm3.Simulation(w, precision="f64", adjoint=True)
    s0 = sim.get_state()
    fl = torch.as_tensor(w.solid == 0, device=s0.device)
    tgt = torch.as_tensor(target, device=s0.device)

    def loss_from(state):
        sim.set_state(state)
        sim.step(steps)
        C = rollout.phase_fields(sim.densities(), [w])[0]
        return float((((C - tgt) ** 2) * fl).sum())

    # lambda_0 by the adjoint, stepping back through stored states
    states = []
    sim.set_state(s0)
    for _ in range(steps):
        states.append(sim.get_state())
        sim.step(1)
    rho = sim.densities().requires_grad_(True)
    C = rollout.phase_fields(rho, [w])[0]
    (((C - tgt) ** 2) * fl).sum().backward()
    lam = torch.empty_like(s0)
    lam2 = torch.full_like(s0, 255)  # NaN everywhere: every node entry must be written
    sim.adjoint_seed(rho.grad, lam)
    for t in reversed(range(steps)):
        sim.adjoint_step(states[t], lam, lam2)
        lam, lam2 = lam2, lam
    lam0 = lam.view(torch.float64)
    mask = torch.as_tensor(_fluid_state_mask(w), device=s0.device)
    smask = torch.as_tensor(_fluid_state_mask(w, solid=True), device=s0.device)
    for buf in (lam0, lam2.view(torch.float64)):  # lambda_0, and lambda_1 in the buffer that began as NaN
        assert bool(torch.isfinite(buf[mask | smask]).all())
        assert float(buf[smask].abs().max()) == 0.0  # entries at solid nodes are zero
    n9 = 9 * (lam0.numel() // 12)
    gen = torch.Generator(device="cpu").manual_seed(5)
    for part, sl in (("distributions", slice(0, n9)), ("densities", slice(n9, None))):
        # random direction at fluid entries; density entries scaled by their value
        delta = torch.zeros_like(lam0)
        r = torch.randn(lam0.numel(), generator=gen, dtype=torch.float64).to(s0.device)
        scale = torch.where(torch.arange(lam0.numel(), device=s0.device) < n9,
                            torch.ones_like(lam0), s0.view(torch.float64).abs())
        delta[sl] = (r * mask * scale)[sl]
        eps = 1e-6
        sp = (s0.view(torch.float64) + eps * delta).contiguous().view(torch.uint8)
        sm = (s0.view(torch.float64) - eps * delta).contiguous().view(torch.uint8)
        fd = (loss_from(sp) - loss_from(sm)) / (2 * eps)
        ad = float((lam0[mask] * delta[mask]).sum())
        print(f"directional ({part}): adjoint {ad:.12e} fd {fd:.12e}", flush=True)
        assert abs(ad - fd) <= 1e-6 * abs(fd)
    sim.close()


# Tolerance of the inverse-problem check per precision, against the oracle's finest difference
# quotient (h/80: 6.25e-4 degree, 1.25e-5 sigma).  L(p) has kinks within a few thousandths of a
# degree of the gradient point, so the quotients at h/10, h/20 and h/40 still straddle some (they
# differ from each other by up to 1 %) while at h/80 they are local: the FP64 adjoint meets them to
# ~1e-4 (the quotient's own resolution of the remaining curvature); FP32 differs from FP64 by its
# forward error (~1e-5 in rho_k after 4000 steps).
INVERSE_TOL = {"f64": 5e-4, "f32": 1e-3}


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_inverse_problem_vs_oracle_fd(precision):
    torch, lbm3, rollout = _mods()
    path = os.path.join(HERE, "golden", "adjoint_fd.json")
    gold = json.load(open(path))
    w = W.inverse_problem(hidden=False)
    wt = W.inverse_problem(hidden=True)
    steps = gold["steps"]
    po.set_threads(po.max_threads())
    target = oracle_C(wt, steps)
    print("target done", flush=True)
    L, g = gpu_grad(torch, lbm3, rollout, w, steps, target, precision, every=gold["checkpoint_every"])
    for scale, fd in gold["fd"].items():
        e = np.abs(g - np.array(fd["grad_fd"])) / np.abs(np.array(fd["grad_fd"]))
        print(f"{precision}: rel err against the oracle difference at h x {scale}: {e}", flush=True)
    g_fd = np.array(gold["fd"]["0.0125"]["grad_fd"])
    err = np.abs(g - g_fd) / np.abs(g_fd)
    print(f"loss gpu {precision} {L:.10e} oracle {gold['loss']:.10e}", flush=True)
    print(f"adjoint {g}\noracle fd (h/80) {g_fd}", flush=True)
    assert abs(L - gold["loss"]) <= (1e-9 if precision == "f64" else 1e-4) * gold["loss"]
    assert err.max() <= INVERSE_TOL[precision]


def _density_part(lam, ws, d):
    """The density planes of domain d of a state-layout FP64 buffer: [3, ny, nx]."""
    import torch
    v = lam.view(torch.float64)
    planes = [((w.nx + 63) // 64 * 64) * (w.ny + 4) for w in ws]
    tplane, base = sum(planes), sum(planes[:d])
    w = ws[d]
    pitch = (w.nx + 63) // 64 * 64
    out = []
    for k in range(3):
        o = 9 * tplane + 3 * base + k * planes[d]
        out.append(v[o:o + planes[d]].reshape(w.ny + 4, pitch)[2:2 + w.ny, :w.nx])
    return torch.stack(out).cpu().numpy()


def test_loss_seed_vs_numpy():
    """lbm3_loss_seed (the device loss of the inverse problem and its lambda_T) through the C ABI:
    the loss against numpy on the GPU's own fields (1e-12) and on the oracle's fields (1e-10), and
    lambda_T against dL/drho_k = (2/rho)[(C_k - C*_k) - sum_l C_l (C_l - C*_l)] written out in numpy
    (1e-12), for two batched domains."""
    torch, lbm3, rollout = _mods()
    cases = small_cases()
    ws = [cases["walls_circle"], cases["swap13"]]
    steps = 20
    targets = [oracle_C(target_setup(w), steps) for w in ws]
    print("loss seed: 2 domains, f64, 20 steps", flush=True)
    sim = lbm3.Simulation(ws, precision="f64", adjoint=True)
    sim.step(steps)
    tgt = torch.cat([torch.as_tensor(t).reshape(-1) for t in targets]).to(sim.device)
    lam = torch.empty(sim.state_bytes(), dtype=torch.uint8, device=sim.device)
    loss = sim.loss_seed(tgt, lam).cpu().numpy()
    for d, (w, t) in enumerate(zip(ws, targets)):
        rho = sim.fields(d, velocity=False, force=False)["rho"].cpu().numpy()
        fl = w.solid == 0
        tot = np.where(fl, rho.sum(0), 1.0)
        C = np.where(fl, rho / tot, 0.0)
        L_np = mismatch(C, t, w.solid)
        L_or = mismatch(oracle_C(w, steps), t, w.solid)
        print(f"domain {d}: loss device {loss[d]:.16e} numpy {L_np:.16e} oracle {L_or:.16e}", flush=True)
        assert abs(loss[d] - L_np) <= 1e-12 * L_np
        assert abs(loss[d] - L_or) <= 1e-10 * L_or
        dC = C - t
        m = (C * dC).sum(0)
        lam_np = np.where(fl, 2.0 * (dC - m) / tot, 0.0)
        got = _density_part(lam, ws, d)
        err = np.abs(got - lam_np).max() / np.abs(lam_np).max()
        print(f"domain {d}: lambda_T rel err {err:.3e}", flush=True)
        assert err <= 1e-12
    v = lam.view(torch.float64)
    n9 = 9 * (v.numel() // 12)
    assert float(v[:n9].abs().max()) == 0.0
    sim.close()


def test_rollout_loss_gradient_equals_rollout_gradient():
    """rollout_loss (device loss, lambda_T from lbm3_loss_seed) and rollout + a torch loss give
    the same parameter gradient; a weight on the loss scales it."""
    torch, lbm3, rollout = _mods()
    w = small_cases()["walls_circle"]
    steps = 16
    target = oracle_C(target_setup(w), steps)
    sim = lbm3.Simulation(w, precision="f64", adjoint=True)
    s0 = sim.get_state()
    p = rollout.params_of([w]).requires_grad_(True)
    rho = rollout.rollout(p, sim, steps, s0, 6)
    C = rollout.phase_fields(rho, [w])[0]
    fl = torch.as_tensor(w.solid == 0, device=C.device)
    tg = torch.as_tensor(target, device=C.device)
    (((C - tg) ** 2) * fl).sum().backward()
    g_ref = p.grad.clone()
    p2 = rollout.params_of([w]).requires_grad_(True)
    L = rollout.rollout_loss(p2, sim, steps, s0, tg.reshape(-1), 6)
    (2.5 * L.sum()).backward()
    err = (p2.grad / 2.5 - g_ref).abs().max() / g_ref.abs().max()
    print(f"rollout_loss vs rollout gradient: rel err {float(err):.3e}", flush=True)
    assert float(err) <= 1e-12
    sim.close()


def test_rollout_backward_uses_its_own_parameters():
    """Two rollouts at different parameters on one Simulation, then the first one's backward:
    its gradient equals that of a rollout at those parameters alone, the Simulation keeps the
    parameters it was last given, and the gradient comes back on the parameters' device."""
    torch, lbm3, rollout = _mods()
    w = small_cases()["walls_circle"]
    steps = 12
    target = torch.as_tensor(oracle_C(target_setup(w), steps))
    fl = torch.as_tensor(w.solid == 0)
    sim = lbm3.Simulation(w, precision="f64", adjoint=True)
    s0 = sim.get_state()

    def loss(rho):
        C = rollout.phase_fields(rho, [w])[0]
        return (((C - target.to(C.device)) ** 2) * fl.to(C.device)).sum()

    pa = rollout.params_of([w]).to(sim.device).requires_grad_(True)
    loss(rollout.rollout(pa, sim, steps, s0, 5)).backward()
    g_alone = pa.grad.clone()
    assert pa.grad.device == pa.device
    p1 = rollout.params_of([w]).to(sim.device).requires_grad_(True)
    p2 = (rollout.params_of([w]) + torch.tensor([[4.0, -3.0, 0.0, 0.0, 0.0]], dtype=torch.float64)).to(sim.device)
    rho1 = rollout.rollout(p1, sim, steps, s0, 5)
    rollout.rollout(p2.requires_grad_(True), sim, steps, s0, 5)
    loss(rho1).backward()
    err = (p1.grad - g_alone).abs().max() / g_alone.abs().max()
    print(f"gradient after an interleaved rollout: rel err {float(err):.3e}", flush=True)
    assert float(err) <= 1e-12  # (the adjoint's float atomics may reorder sums)
    np.testing.assert_array_equal(sim.params[0], p2.detach().cpu().numpy()[0])
    sim.close()
