"""Differentiable rollout of the three-phase update (arXiv:2102.04709, Sec. II) behind
torch.autograd.Function, with checkpoint-and-recompute.

`rollout(params, sim, steps, init_state, every)` runs `steps` time steps of every domain of
`sim` (an lbm3.Simulation created with adjoint=True) from `init_state` with the wetting and
tension parameters `params` ([n_domains, 5]: theta13, theta23 in degrees, sigma12, sigma13,
sigma23) and returns the partial densities at the last step (flat, [3][ny][nx] per domain,
zero at solid nodes).  Its backward pass gives dL/dparams for any loss L of those densities:
the forward keeps a state checkpoint every `every` steps; the backward replays each block from
its checkpoint, keeping the block's states, and runs the hand-written adjoint step
(lbm3_adjoint_step) backwards through it.  Device memory: (steps / every + every) states.
"""
from __future__ import annotations

import numpy as np
import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, sim, steps, init_state, every):
        p = params.detach().to("cpu", torch.float64).numpy().reshape(sim.n, 5)
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
        out = sim.densities()
        ctx.sim, ctx.steps, ctx.every, ctx.ckpts = sim, int(steps), int(every), ckpts
        ctx.param_dtype = params.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out):
        sim, steps, every = ctx.sim, ctx.steps, ctx.every
        nb = sim.state_bytes()
        lam = torch.empty(nb, dtype=torch.uint8, device=sim.device)
        lam2 = torch.empty_like(lam)
        sim.adjoint_seed(grad_out, lam)
        resume = sim.get_state()
        block = torch.empty((min(every, steps), nb), dtype=torch.uint8, device=sim.device)
        for b in reversed(range(len(ctx.ckpts))):
            k = min(every, steps - b * every)
            sim.set_state(ctx.ckpts[b])
            for t in range(k):
                sim.get_state(out=block[t])
                if t + 1 < k:
                    sim.step(1)
            for t in reversed(range(k)):
                sim.adjoint_step(block[t], lam, lam2)
                lam, lam2 = lam2, lam
        sim.set_state(resume)
        grad = torch.as_tensor(sim.adjoint_grad(), dtype=ctx.param_dtype).reshape(sim.n, 5)
        ctx.ckpts = None
        return grad, None, None, None, None


def rollout(params: torch.Tensor, sim, steps: int, init_state: torch.Tensor, every: int = 100) -> torch.Tensor:
    return _Rollout.apply(params, sim, steps, init_state, every)


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
