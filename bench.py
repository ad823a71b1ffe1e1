"""Throughput of the three-phase colour-gradient D2Q9 step on one MI355X.

Headline: the 400 x 400 Janus-droplet-on-cylinder workload (interpolated bounce-back on the
cylinder, wetting fill, sigma 0.005, angles 90/90, viscosities 0.05/0.1/0.2) in FP32 with
shifted storage, advanced with hipGraph replays of 100-step blocks; MLUPS counts all nx*ny
nodes.  The same JSON line carries the FP64 and FP16-storage variants, the x10 scale-up of the
workload (4000 x 4000, 1.5 GB of FP32 state, so HBM rather than the 256 MB Infinity Cache sets
the bound), the 96-domain batched pillar sweep in one launch per step, the roofline of the fused
kernel from HIP events on its own stream, the adjoint step and the checkpointed forward +
backward rollout on the 512 x 256 inverse problem (FP32 and FP64), the FP32 adjoint step on the
4000 x 4000 workload, and the FP64 CPU oracle timed on a bounded sample (about 10-20 s).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-extra] [--skip-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the fused kernel from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB
# per dispatch), scaled by what the counters read for a 1 GiB device copy in the same process
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); summaries and commands in profiles/.  Keyed by workload,
# precision and kernel configuration, valid for the kernel sources with the given digest only.
KERNEL_SOURCES = ("lbm3_kernels.hip", "lbm3_device.h", "lbm3_internal.h", "lbm3_kernels.h", "lbm3_adjoint.h")
TRAFFIC = {
    "digest": "09d76c66367a9433",
    ('cylinder_janus', 400, 'f32', (3, 16, 16)): (4478.0 * 2.0 + 6969.0 * 1.0) * 1024,
    ('cylinder_janus_x10', 4000, 'f32', (3, 64, 8)): (363611.0 * 2.0 + 696999.0 * 1.0) * 1024,
    ('cylinder_janus_x10', 4000, 'f16', (3, 64, 8)): (233596.3 * 2.0 + 435784.1 * 1.0) * 1024,
}


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_04709_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(w, precision, config):
    if config is None or kernel_digest() != TRAFFIC["digest"]:
        return None
    v = TRAFFIC.get((w.name, w.nx, precision, tuple(config)))
    return None if v is None else int(v)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_run(sim, steps, warmup):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def roofline(sim, launches=50, traffic=None):
    ms_fill, ms_step = sim.kernel_times(launches)
    nodes = sim.query(1)
    bpl = sim.query(0)
    achieved = bpl * nodes / (ms_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "step_fused", "bytes_per_lup": bpl, "lups_per_launch": int(nodes),
            "ms_per_launch": round(ms_step, 5), "fill_kernel_ms_per_launch": round(ms_fill, 5)}


def graph_block_for(steps, preferred):
    """Steps per captured graph: the preferred block, or less so that the timed steps replay at
    least two graphs (lbm3_step replays a graph only for whole blocks)."""
    if preferred <= 0:
        return 0
    return max(2, min(preferred, (steps // 2) // 2 * 2))


def measure(workloads_, precision, steps, warmup, graph=100, config=None, persistent=0):
    """config = (kernel, tile_x, tile_y) as lbm3_autotune returns it; None runs the autotuner."""
    from paper_2102_04709_amd import lbm3
    graph = graph_block_for(steps, graph)
    if config is None:
        sim = lbm3.Simulation(workloads_, precision=precision, graph_block_steps=graph,
                              persistent_blocks=persistent)
        tile = sim.autotune(20)  # 20 launches per candidate: a stable pick between close configurations
    else:
        k, tx, ty = config
        sim = lbm3.Simulation(workloads_, precision=precision, graph_block_steps=graph, kernel=int(k),
                              tile=(tx, ty) if k in (0, 3) else (0, ty), persistent_blocks=persistent)
        tile = tuple(config)
    sim.step(warmup)
    g0 = sim.query(9)
    dt = timed_run(sim, steps, 0)
    replays = int(sim.query(9) - g0)
    nodes = sim.query(1)
    traffic = traffic_for(workloads_[0], precision, tile) if len(workloads_) == 1 else None
    res = {"mlups": round(nodes * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 5),
           "tile": list(tile) if tile else None, "graph_block_steps": graph,
           "graph_replays_timed": replays, "steps_in_graphs": replays * graph,
           "persistent_blocks": persistent, "roofline": roofline(sim, traffic=traffic)}
    sim.close()
    return res, dt


def measure_adjoint(w, precision, steps=40, rollout_steps=400, every=100):
    """Adjoint step throughput (lbm3_adjoint_step over stored forward states, HIP events on the
    library's stream) and the checkpointed forward + backward rollout of `rollout_steps` steps.
    Algorithmic bytes per node of one adjoint step: the forward state s_t read, lambda_{t+1}
    read and lambda_t written, each 9 distributions + 3 densities."""
    import torch
    from paper_2102_04709_amd import lbm3, rollout
    sim = lbm3.Simulation([w], precision=precision, adjoint=True)
    sim.step(100)
    nb = sim.state_bytes()
    states = torch.empty((steps, nb), dtype=torch.uint8, device=sim.device)
    for t in range(steps):
        sim.get_state(out=states[t])
        sim.step(1)
    gen = torch.Generator(device="cpu").manual_seed(1)
    g = torch.randn(3 * w.nx * w.ny, generator=gen, dtype=torch.float64).to(sim.device)
    lam, lam2 = torch.empty(nb, dtype=torch.uint8, device=sim.device), torch.empty(nb, dtype=torch.uint8, device=sim.device)
    sim.adjoint_seed(g, lam)
    for t in reversed(range(min(5, steps))):
        sim.adjoint_step(states[t], lam, lam2)
        lam, lam2 = lam2, lam
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(sim.stream)
    for t in reversed(range(steps)):
        sim.adjoint_step(states[t], lam, lam2)
        lam, lam2 = lam2, lam
    ev1.record(sim.stream)
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    nodes = w.nx * w.ny
    bpl = 3 * (9 * (8 if precision == "f64" else 4) + 3 * (8 if precision == "f64" else 4))
    achieved = bpl * nodes / (ms * 1e-3) / 1e9
    res = {"mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "adjoint step (all kernels of lbm3_adjoint_step)", "bytes_per_lup": bpl,
                        "lups_per_launch": nodes}}
    if rollout_steps <= 0:
        sim.close()
        return res
    # checkpointed rollout: forward with checkpoints, backward with recompute and adjoint steps
    s0 = sim.get_state()
    params = rollout.params_of([w]).requires_grad_(True)
    (rollout.rollout(params, sim, every, s0, every) * g).sum().backward()  # untimed warm-up
    params.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho = rollout.rollout(params, sim, rollout_steps, s0, every)
    (rho * g).sum().backward()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["rollout"] = {"steps": rollout_steps, "checkpoint_every": every, "seconds": round(dt, 3),
                      "mlups_forward_plus_backward": round(nodes * rollout_steps / dt / 1e6, 1)}
    sim.close()
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, steps, threads):
    from oracle import pyoracle as po
    po.set_threads(threads)
    o = po.Oracle(w)
    o.step(1)  # untimed: thread pool start and first touch of the arrays
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return w.nodes * steps / dt / 1e6, dt


def cpu_baseline(w, budget_s=20.0, full=True):
    """The FP64 oracle (plain, untuned) on the host cores.  The headline value is its MLUPS on the
    headline workload with all threads, on a bounded sample; with full=True the line also carries
    the per-configuration samples of the baseline plan at 1 thread and at all threads (steps cut so
    the whole leg stays within about a minute) and the wall time of the adjoint's finite-difference
    set extrapolated from the measured inverse-problem rate."""
    from oracle import pyoracle as po
    from paper_2102_04709_amd import workloads as W
    threads = po.max_threads()
    rate0, dt0 = _oracle_rate(w, 20, threads)
    n = max(1, min(20000, int(budget_s / max(dt0 / 20, 1e-6))))
    rate, dt = _oracle_rate(w, n, threads)
    out = {"value": round(rate, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{w.name} {w.nx}x{w.ny}, FP64 oracle, {n} steps after 1 untimed step, {dt:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if not full:
        return out
    sweep = W.pillar_sweep()
    by_size = sorted(sweep, key=lambda v: v.nodes)
    plan = [("flat_janus_120x60 (full 2000 steps)", W.flat_janus(), 2000, 200),
            ("cylinder_janus_400x400", w, 200, 10),
            ("capillary_intrusion_1024x64 ratio 100", W.capillary_intrusion(ratio=100.0), 200, 20),
            ("pillar sweep, smallest domain", by_size[0], 100, 10),
            ("pillar sweep, 2nd smallest domain", by_size[1], 100, 10),
            ("pillar sweep, 2nd largest domain", by_size[-2], 100, 5),
            ("pillar sweep, largest domain", by_size[-1], 100, 5),
            ("inverse problem 512x256", W.inverse_problem(), 100, 10)]
    rows = []
    for name, wk, steps_all, steps_one in plan:
        r_all, t_all = _oracle_rate(wk, steps_all, threads)
        r_one, t_one = _oracle_rate(wk, steps_one, 1)
        rows.append({"config": name, "nodes": wk.nodes, "steps_all_threads": steps_all,
                     "mlups_all_threads": round(r_all, 3), "steps_1_thread": steps_one,
                     "mlups_1_thread": round(r_one, 3), "seconds": round(t_all + t_one, 2)})
    po.set_threads(threads)
    inv = rows[-1]
    fd_lup = 2 * 4 * 5 * 4000 * inv["nodes"] + 2 * 4000 * inv["nodes"]
    out["plan"] = rows
    out["fd_set_wall_s_extrapolated"] = round(fd_lup / (inv["mlups_all_threads"] * 1e6), 1)
    out["fd_set_note"] = ("42 oracle runs of 4000 steps (loss, target, 5 parameters x 2 signs x 4 steps h, h/2, "
                          "h/10, h/80) at the measured all-thread rate")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-quick", action="store_true", help="only the headline sample of the CPU baseline")
    ap.add_argument("--only", default=None,
                    help="run one workload (cylinder_400_f32|f64|f16, cylinder_4000_f32|f64|f16, "
                         "pillar_sweep_96_f32, adjoint_512_f32|f64, adjoint_4000_f32) and print its measurement")
    ap.add_argument("--config", default=None,
                    help="fixed kernel configuration 'KERNEL,TX,TY' for --only, as the autotuner reports "
                         "it (0/3 = tiles TX x TY of 256/512 threads, 1/2 = strips of 128/256 threads "
                         "with TY rows)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2102_04709_amd import workloads as W

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device-to-device copies")
    if args.only:
        name = args.only
        if name.startswith("adjoint_512"):
            r = measure_adjoint(W.inverse_problem(), name.rsplit("_", 1)[1])
            print(json.dumps({"workload": name, **r}), flush=True)
            return
        if name.startswith("adjoint_4000"):
            r = measure_adjoint(W.cylinder_janus_hbm(10), name.rsplit("_", 1)[1], steps=24, rollout_steps=0)
            print(json.dumps({"workload": name, **r}), flush=True)
            return
        if name.startswith("pillar_sweep"):
            ws, graph = W.pillar_sweep(), 10
        elif name.startswith("cylinder_4000"):
            ws, graph = [W.cylinder_janus_hbm(10)], 10
        else:
            ws, graph = [W.cylinder_janus()], 100
        config = tuple(int(v) for v in args.config.split(",")) if args.config else None
        r, _ = measure(ws, name.rsplit("_", 1)[1], args.steps, args.warmup, graph=graph, config=config)
        print(json.dumps({"workload": name, **r}), flush=True)
        return
    w = W.cylinder_janus()
    log(f"headline: {w.name} {w.nx}x{w.ny} f32, steps={args.steps} warmup={args.warmup}")
    head, dt = measure([w], "f32", args.steps, args.warmup)
    out = {
        "metric": "MLUPS and % HBM roofline, FP32 vs FP64 step, batched sweep, adjoint step",
        "value": head["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cylinder_janus_400x400", "nx": 400, "ny": 400,
                   "precision": "f32 compute, f32 shifted storage",
                   "graph_block_steps": head["graph_block_steps"],
                   "graph_replays_timed": head["graph_replays_timed"],
                   "tile": head["tile"], "parallelism": "1 GPU"},
        "roofline": head["roofline"],
    }
    if not args.skip_extra:
        extra = {}
        for p in ("f64", "f16"):
            log(f"variant: {w.name} {p}")
            r, _ = measure([w], p, args.steps // 2, args.warmup // 2)
            extra[f"cylinder_400_{p}"] = r
        hbm = W.cylinder_janus_hbm(10)
        for p in ("f32", "f64", "f16"):
            log(f"variant: {hbm.name} {p}")
            r, _ = measure([hbm], p, 100, 10, graph=10)
            extra[f"cylinder_4000_{p}"] = r
        log("variant: batched pillar sweep (96 domains)")
        sweep = W.pillar_sweep()
        r, _ = measure(sweep, "f32", 100, 10, graph=10)
        r["domains"] = len(sweep)
        extra["pillar_sweep_96_f32"] = r
        log("variant: batched pillar sweep, persistent launch (one work-group loop per slot)")
        cfg = tuple(r["tile"])
        slots = 256 * (6 if cfg[0] == 0 else 3)  # the work-groups one round of the chip holds
        rp, _ = measure(sweep, "f32", 100, 10, graph=10, config=cfg, persistent=slots)
        rp["domains"] = len(sweep)
        extra["pillar_sweep_96_f32_persistent"] = rp
        for p in ("f32", "f64"):
            log(f"variant: adjoint step, inverse problem 512x256 {p}")
            extra[f"adjoint_512_{p}"] = measure_adjoint(W.inverse_problem(), p)
        log("adjoint step at HBM scale: 4000x4000 cylinder, f32")
        extra["adjoint_4000_f32"] = measure_adjoint(W.cylinder_janus_hbm(10), "f32", steps=24, rollout_steps=0)
        out["variants"] = extra
        out["roofline_hbm"] = extra["cylinder_4000_f32"]["roofline"]
    if not args.skip_cpu:
        log("cpu baseline: oracle")
        out["cpu_baseline"] = cpu_baseline(w, full=not args.cpu_quick)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
