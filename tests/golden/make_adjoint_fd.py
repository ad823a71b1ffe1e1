"""Writes adjoint_fd.json: central finite differences of the FP64 oracle for the inverse
problem (512 x 256, twelve pillars, compound droplet; Sec. III set-ups), the reference values
of the adjoint's gradient test.

Loss: L = sum over fluid nodes and fluids k of (C_k - C*_k)^2 after `steps` steps from the
initial fields, where C* is the oracle's result at the hidden parameters (theta13, theta23) =
(40, 110) degrees and its tensions.  Parameters p = (theta13, theta23 in degrees, sigma12,
sigma13, sigma23); steps h = 0.05 degree for the angles and 1e-3 sigma for the tensions, and
h/2, h/10 and h/80.  L(p) is only piecewise smooth (the clamps of Eq. 10 and 14, the max/min of
Eq. 22, the discrete crossings of the characteristic lines), so the larger steps average the slope
over kinks; the test compares with the finest, h/80.
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
# difference steps as fractions of h = (0.05 degree, 0.05 degree, 1e-3 sigma); L(p) is only
# piecewise smooth and has kinks within a few thousandths of a degree of the gradient point, so the
# finest step is the one the adjoint is compared with
SCALES = (1.0, 0.5, 0.1, 0.0125)


def phase(w):
    o = po.Oracle(w)
    o.step(STEPS)
    r = o.rho()
    fl = w.solid == 0
    return np.where(fl, r / np.where(fl, r.sum(0), 1.0), 0.0)


def loss(C, target, solid):
    return float(((C - target)[:, solid == 0] ** 2).sum())


_TARGET = None


def _init(threads, target):
    global _TARGET
    po.set_threads(threads)
    _TARGET = target


def _loss_at(p):
    w = W.inverse_problem(hidden=False)
    wk = w.with_params(theta_deg=(p[0], p[1]), sigma=(p[2], p[3], p[4]))
    return loss(phase(wk), _TARGET, w.solid)


def main():
    obuild.build()
    t0 = time.time()
    # oracle runs in parallel processes of a few threads each (the runs are memory bound)
    workers = max(1, min(int(os.environ.get("FD_WORKERS", "3")), os.cpu_count() or 1))
    threads = max(1, ((os.cpu_count() or 1) - (1 if workers > 1 else 0)) // workers)
    po.set_threads(po.max_threads())
    w = W.inverse_problem(hidden=False)
    target = phase(W.inverse_problem(hidden=True))
    p0 = np.array([*w.theta_deg, *w.sigma])
    h0 = np.array([0.05, 0.05, *(1e-3 * np.array(w.sigma))])
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd.json")
    # differences already in the file (same steps and parameters) are kept; only new scales run
    old = {}
    if os.path.exists(out_path):
        prev = json.load(open(out_path))
        if prev.get("steps") == STEPS and np.allclose(prev.get("params", []), p0):
            old = prev["fd"]
    scales = tuple(sc for sc in SCALES if str(sc) not in old)
    points = [p0.copy()]
    for scale in scales:
        for k in range(5):
            for sgn in (1.0, -1.0):
                p = p0.copy()
                p[k] += sgn * h0[k] * scale
                points.append(p)
    import multiprocessing as mp
    # spawned, not forked: the parent has started OpenMP threads, which a forked child cannot use
    with mp.get_context("spawn").Pool(workers, initializer=_init, initargs=(threads, target)) as pool:
        vals = []
        for n, v in enumerate(pool.imap(_loss_at, points)):
            vals.append(v)
            print(f"run {n + 1}/{len(points)}: loss {v:.12e} ({time.time() - t0:.0f} s)", flush=True)
    L0 = vals[0]
    fds = dict(old)
    i = 1
    for scale in scales:
        h = h0 * scale
        g = []
        for k in range(5):
            g.append((vals[i] - vals[i + 1]) / (2 * h[k]))
            i += 2
        fds[str(scale)] = {"h": h.tolist(), "grad_fd": g}
        print(f"h x {scale}: {g}", flush=True)
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
    out["fd"] = {str(sc): fds[str(sc)] for sc in SCALES}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
