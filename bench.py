"""Throughput of the three-phase colour-gradient D2Q9 step on one MI355X.

Headline: the 400 x 400 Janus-droplet-on-cylinder workload (interpolated bounce-back on the
cylinder, wetting fill, sigma 0.005, angles 90/90, viscosities 0.05/0.1/0.2) in FP32 with
shifted storage, advanced with hipGraph replays of 100-step blocks; MLUPS counts all nx*ny
nodes.  The same JSON line carries the FP64 and FP16-storage variants, the x10 scale-up of the
workload (4000 x 4000, 1.5 GB of FP32 state, so HBM rather than the 256 MB Infinity Cache sets
the bound), the 96-domain batched pillar sweep in one launch per step, the roofline of the fused
kernel from HIP events on its own stream, and the FP64 CPU oracle timed on a bounded sample.

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


def roofline(sim, launches=50):
    ms_fill, ms_step = sim.kernel_times(launches)
    nodes = sim.query(1)
    bpl = sim.query(0)
    achieved = bpl * nodes / (ms_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "step_fused", "bytes_per_lup": bpl, "lups_per_launch": int(nodes),
            "ms_per_launch": round(ms_step, 5), "fill_kernel_ms_per_launch": round(ms_fill, 5)}


def measure(workloads_, precision, steps, warmup, graph=100, tile=None):
    from paper_2102_04709_amd import lbm3
    sim = lbm3.Simulation(workloads_, precision=precision, graph_block_steps=graph, tile=tile)
    tile = sim.autotune(3) if tile is None else tile
    dt = timed_run(sim, steps, warmup)
    nodes = sim.query(1)
    res = {"mlups": round(nodes * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 5),
           "tile": list(tile) if tile else None, "roofline": roofline(sim)}
    sim.close()
    return res, dt


def cpu_baseline(w, budget_s=15.0):
    from oracle import pyoracle as po
    threads = po.max_threads()
    po.set_threads(threads)
    o = po.Oracle(w)
    t0 = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t0) / 2
    n = max(1, min(2000, int(budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(w.nodes * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{w.name} {w.nx}x{w.ny}, FP64 oracle, {n} steps after 2 warm-up steps, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--skip-extra", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--only", default=None,
                    help="run one workload (cylinder_400_f32|f64|f16, cylinder_4000_f32|f64|f16, "
                         "pillar_sweep_96_f32) and print its measurement")
    ap.add_argument("--tile", default=None, help="fixed tile 'TX,TY' for --only (skips the autotuner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
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
        if name.startswith("pillar_sweep"):
            ws, graph = W.pillar_sweep(), 10
        elif name.startswith("cylinder_4000"):
            ws, graph = [W.cylinder_janus_hbm(10)], 10
        else:
            ws, graph = [W.cylinder_janus()], 100
        tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
        r, _ = measure(ws, name.rsplit("_", 1)[1], args.steps, args.warmup, graph=graph, tile=tile)
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
                   "precision": "f32 compute, f32 shifted storage", "graph_block_steps": 100,
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
        out["variants"] = extra
        out["roofline_hbm"] = extra["cylinder_4000_f32"]["roofline"]
    if not args.skip_cpu:
        log("cpu baseline: oracle")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
