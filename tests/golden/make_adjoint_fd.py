"""Writes adjoint_fd.json: central finite differences of the FP64 oracle for the inverse
problem (512 x 256, twelve pillars, compound droplet; Sec. III set-ups), the reference values
of the adjoint's gradient test.

Loss: L = sum over fluid nodes and fluids k of (C_k - C*_k)^2 after `steps` steps from the
initial fields, where C* is the oracle's result at the hidden parameters (theta13, theta23) =
(40, 110) degrees and its tensions.  Parameters p = (theta13, theta23 in degrees, sigma12,
sigma13, sigma23); steps h = 0.05 degree for the angles and 1e-3 sigma for the tensions, and
h/2 and h/10.  L(p) is only piecewise smooth (the clamps of Eq. 10 and 14, the max/min of
Eq. 22), so the larger steps average the slope over kinks; the test compares with h/10.
Calls only the oracle.  Run from the repository root:  python tests/golden/make_adjoint_fd.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import build as obuild  # noqa: E402
from oracle import pyoracle as po  # noqa: E402
from paper_2102_04709_amd import workloads as W  # noqa: E402

STEPS = 4000


def phase(w):
    o = po.Oracle(w)
    o.step(STEPS)
    r = o.rho()
    fl = w.solid == 0
    return np.where(fl, r / np.where(fl, r.sum(0), 1.0), 0.0)


def loss(C, target, solid):
    return float(((C - target)[:, solid == 0] ** 2).sum())


def main():
    obuild.build()
    po.set_threads(po.max_threads())
    t0 = time.time()
    w = W.inverse_problem(hidden=False)
    target = phase(W.inverse_problem(hidden=True))
    L0 = loss(phase(w), target, w.solid)
    print(f"loss {L0:.12e} ({time.time() - t0:.0f} s)", flush=True)
    p0 = np.array([*w.theta_deg, *w.sigma])
    h0 = np.array([0.05, 0.05, *(1e-3 * np.array(w.sigma))])
    fds = {}
    for scale in (1.0, 0.5, 0.1):
        h = h0 * scale
        g = []
        for k in range(5):
            v = []
            for sgn in (1.0, -1.0):
                p = p0.copy()
                p[k] += sgn * h[k]
                wk = w.with_params(theta_deg=(p[0], p[1]), sigma=(p[2], p[3], p[4]))
                v.append(loss(phase(wk), target, w.solid))
            g.append((v[0] - v[1]) / (2 * h[k]))
            print(f"h x {scale}: param {k}: {g[-1]:.10e} ({time.time() - t0:.0f} s)", flush=True)
        fds[str(scale)] = {"h": h.tolist(), "grad_fd": g}
    out = {
        "what": "central differences of the FP64 oracle's phase-field mismatch loss, inverse problem 512x256",
        "steps": STEPS,
        "checkpoint_every": 100,
        "params": p0.tolist(),
        "params_names": ["theta13_deg", "theta23_deg", "sigma12", "sigma13", "sigma23"],
        "hidden_params": [*W.inverse_problem(hidden=True).theta_deg, *W.inverse_problem(hidden=True).sigma],
        "loss": L0,
        "fd": fds,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
