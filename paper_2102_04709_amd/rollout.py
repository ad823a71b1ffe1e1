"""Differentiable rollout of the three-phase update (arXiv:2102.04709, Sec. II) behind
torch.autograd.Function, with checkpoint-and-recompute.

`rollout(params, sim, steps, init_state, every)` runs `steps` time steps of every domain of
`sim` (an lbm3.Simulation created with adjoint=True) from `init_state` with the wetting and
tension parameters `params` ([n_domains, 5]: theta13, theta23 in degrees, sigma12, sigma13,
sigma23) and returns the partial densities at the last step (flat, [3][ny][nx] per domain,
zero at solid nodes).  Its backward pass gives dL/dparams for any loss L of those densities.

`rollout_loss(params, sim, steps, init_state, target, every)` returns the phase-field mismatch
loss sum_k sum_fluid (C_k - C*_k)^2 per domain ([n_domains]), formed on the device by
lbm3_loss_seed, which also seeds the backward pass.

Both keep a state checkpoint every `every` steps in the forward pass; the backward pass replays
each block from its checkpoint, keeping the block's states, and runs the hand-written adjoint
step (lbm3_adjoint_step) backwards through it.  Device memory: (steps / every + every) states.
The backward pass runs at the parameters of its own forward pass (whatever the Simulation was
set to in between) and leaves the Simulation's parameters and state as it found them.
"""
from __future__ import annotations

import numpy as np
import torch


def _forward(sim, p, steps, init_state, every):
    for d in range(sim.n):
        sim.set_params(d, p[d, :2], p[d, 2:])
    sim.set_state(init_state)
    ckpts = []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        ckpts.append(sim.get_state())
        sim.step(k)
        done += k
    return ckpts


def _backward(sim, p, steps, every, ckpts, seed):
    """Runs the adjoint through the blocks at parameters p; seed(lam) writes lambda_T.  Returns
    the parameter gradient [n, 5] (float64, CPU) and restores the caller's parameters and state."""
    saved_params = sim.params.copy()
    resume = sim.get_state()
    for d in range(sim.n):
        sim.set_params(d, p[d, :2], p[d, 2:])
    nb = sim.state_bytes()
    lam = torch.empty(nb, dtype=torch.uint8, device=sim.device)
    lam2 = torch.empty_like(lam)
    seed(lam)
    block = torch.empty((min(every, steps), nb), dtype=torch.uint8, device=sim.device)
    for b in reversed(range(len(ckpts))):
        k = min(every, steps - b * every)
        sim.set_state(ckpts[b])
        for t in range(k):
            sim.get_state(out=block[t])
            if t + 1 < k:
                sim.step(1)
        for t in reversed(range(k)):
            sim.adjoint_step(block[t], lam, lam2)
            lam, lam2 = lam2, lam
    grad = sim.adjoint_grad()
    for d in range(sim.n):
        sim.set_params(d, saved_params[d, :2], saved_params[d, 2:])
    sim.set_state(resume)
    return grad


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, sim, steps, init_state, every):
        p = params.detach().to("cpu", torch.float64).numpy().reshape(sim.n, 5).copy()
        ckpts = _forward(sim, p, steps, init_state, every)
        out = sim.densities()
        ctx.sim, ctx.steps, ctx.every, ctx.ckpts, ctx.p = sim, int(steps), int(every), ckpts, p
        ctx.param_dtype, ctx.param_device = params.dtype, params.device
        return out

    @staticmethod
    def backward(ctx, grad_out):
        sim = ctx.sim
        grad = _backward(sim, ctx.p, ctx.steps, ctx.every, ctx.ckpts,
                         lambda lam: sim.adjoint_seed(grad_out, lam))
        ctx.ckpts = None
        g = torch.as_tensor(grad, dtype=ctx.param_dtype).reshape(sim.n, 5).to(ctx.param_device)
        return g, None, None, None, None


class _RolloutLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, sim, steps, init_state, target, every):
        p = params.detach().to("cpu", torch.float64).numpy().reshape(sim.n, 5).copy()
        ckpts = _forward(sim, p, steps, init_state, every)
        scratch = torch.empty(sim.state_bytes(), dtype=torch.uint8, device=sim.device)
        loss = sim.loss_seed(target, scratch)
        ctx.sim, ctx.steps, ctx.every, ctx.ckpts, ctx.p = sim, int(steps), int(every), ckpts, p
        ctx.final = sim.get_state()
        ctx.target = target
        ctx.param_dtype, ctx.param_device = params.dtype, params.device
        return loss.to(params.device)

    @staticmethod
    def backward(ctx, grad_loss):
        sim = ctx.sim
        gl = grad_loss.detach().to("cpu", torch.float64).reshape(-1)

        def seed(lam):
            sim.set_state(ctx.final)
            sim.loss_seed(ctx.target, lam)

        # the domains are independent, so the gradient of sum_d g_d L_d is g_d times the
        # gradient of L_d, domain by domain
        grad = _backward(sim, ctx.p, ctx.steps, ctx.every, ctx.ckpts, seed) * gl.numpy()[:, None]
        ctx.ckpts = ctx.final = None
        g = torch.as_tensor(grad, dtype=ctx.param_dtype).reshape(sim.n, 5).to(ctx.param_device)
        return g, None, None, None, None, None


def rollout(params: torch.Tensor, sim, steps: int, init_state: torch.Tensor, every: int = 100) -> torch.Tensor:
    return _Rollout.apply(params, sim, steps, init_state, every)


def rollout_loss(params: torch.Tensor, sim, steps: int, init_state: torch.Tensor, target: torch.Tensor,
                 every: int = 100) -> torch.Tensor:
    """Per-domain phase-field mismatch loss after `steps` steps (device-side, lbm3_loss_seed);
    target: flat [3][ny][nx] per domain of target mass fractions."""
    return _RolloutLoss.apply(params, sim, steps, init_state, target, every)


def phase_fields(rho_flat: torch.Tensor, workloads):
    """Mass fractions C_k = rho_k / sum_l rho_l per domain ([3, ny, nx], zero at solid nodes)."""
    out, o = [], 0
    for w in workloads:
        n = 3 * w.nx * w.ny
        r = rho_flat[o:o + n].reshape(3, w.ny, w.nx)
        fluid = torch.as_tensor(np.asarray(w.solid) == 0, device=r.device)
        tot = torch.where(fluid, r.sum(0), torch.ones_like(r[0]))
        out.append(torch.where(fluid, r / tot, torch.zeros_like(r)))
        o += n
    return out


def params_of(workloads) -> torch.Tensor:
    return torch.tensor([[*w.theta_deg, *w.sigma] for w in workloads], dtype=torch.float64)
