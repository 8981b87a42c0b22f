"""Throughput of the particle advance on one MI355X.

One step = one pdfmc_step(1): particle kernel (location by neighbour walk,
P1 interpolation, GLM velocity / position / frequency SDEs, IECM mixing,
boundary conditions, scatter of the moments), node statistics, cell means,
Eulerian fields, elliptic-relaxation and projection CG solves, for every
particle of the workload. Inputs are synthetic and resident in HBM before the
timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload channel|cavity|small]
                    [--precision fp32|fp64] [--graph 0|1] [--sort-interval M]

Prints one JSON line (rank 0). Only one GPU is supported: --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (locate+SDE+node stats), FP32/batched vs FP64 at matched error"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import workloads as W
    if name == "channel":
        cfg = W.config_channel()
        return cfg, dict(sort_interval=10)
    if name == "cavity":
        cfg = W.config_cavity()
        return cfg, dict(sort_interval=10)
    if name == "small":
        cfg = W.config_small()
        return cfg, dict(sort_interval=10)
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(prec, ns, n_particles, n_nodes, n_elems):
    """Bytes the particle kernel must move per launch: every particle's state
    read and written once, the node fields read and node sums written once,
    element records and cell tables read/written once."""
    R = 4 if prec == "fp32" else 8
    per_particle = (7 * R + ns * R + 4 + 4 + 1) + (6 * R + ns * R + 4 + 1)
    per_node = 22 * R + 8 * (11 + 2 * ns)
    per_elem = 8 * R + 12 + (8 * ns * R + 8 * (1 + ns) * 8 + 8 * 4 if ns else 0)
    total = n_particles * per_particle + n_nodes * per_node + n_elems * per_elem
    return total, per_particle


def run_gpu(cfg, prec, steps, warmup, opts):
    import torch
    from paper_1006_0549_amd import Sim
    parts = cfg["particles"]
    n = len(parts["x"])
    sim = Sim(prec, "cuda:0")
    cs = sim.add_case(cfg["mesh"], cfg["params"], n)
    ws = sim.bind()
    sim.set_options(sort_interval=opts.get("sort_interval", 0), block_size=256, use_graph=opts.get("graph", False))
    sim.upload(cs, parts)
    sim.init()
    log(f"{prec}: workspace {ws / 2**20:.1f} MiB, {n} particles; warmup {warmup} steps")
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.timing(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    k1_ms, k1_n = sim.timing_read()
    sim.timing(False)
    log(f"{prec}: {steps} steps in {ms:.2f} ms (wall {wall * 1e3:.1f} ms); particle kernel {k1_ms / max(k1_n, 1):.3f} ms/launch")
    stats = sim.stats(cs)
    counters = sim.counters(cs)
    nsn, sn = sim.case_info(cs)
    return dict(ms=ms, k1_ms=k1_ms, k1_n=k1_n, stats=stats, counters=counters, n=n, nsn=nsn, rows=np.unique(sn, return_index=True)[1])


def cpu_baseline(cfg, budget_s=20.0):
    import oracle
    parts = cfg["particles"]
    n = len(parts["x"])
    o = oracle.Oracle()
    oc = o.add_case(cfg["mesh"], cfg["params"])
    o.upload(oc, parts)
    t0 = time.perf_counter()
    o.init()
    log(f"oracle init {time.perf_counter() - t0:.1f} s")
    done, t = 0, 0.0
    while t < budget_s and done < 50:
        t1 = time.perf_counter()
        o.step(1)
        t += time.perf_counter() - t1
        done += 1
        log(f"oracle step {done}: {t:.1f} s")
    return dict(value=n * done / t, unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"{done} full steps of the same workload ({n} particles), single-threaded FP64 C, "
                       f"timed after initialisation")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--sort-interval", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the particle advance is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    t0 = time.perf_counter()
    cfg, opts = workload(args.workload)
    if args.sort_interval is not None:
        opts["sort_interval"] = args.sort_interval
    opts["graph"] = bool(args.graph)
    mesh, params = cfg["mesh"], cfg["params"]
    n = len(cfg["particles"]["x"])
    ns = params["n_scalars"]
    log(f"workload {cfg['name']}: {mesh.n_elems} triangles, {n} particles, {ns} scalars "
        f"(inputs built in {time.perf_counter() - t0:.1f} s)")

    g = run_gpu(cfg, args.precision, args.steps, args.warmup, opts)
    ms_per_step = g["ms"] / args.steps
    value = n * args.steps / (g["ms"] * 1e-3)
    k1_avg_s = g["k1_ms"] / max(g["k1_n"], 1) * 1e-3
    nbytes, per_particle = algorithmic_bytes(args.precision, ns, n, g["nsn"], mesh.n_elems)
    achieved = nbytes / k1_avg_s / 1e9

    extra = {}
    if args.precision == "fp32" and not args.no_fp64_reference:
        r = run_gpu(cfg, "fp64", args.steps, args.warmup, opts)
        rows = r["rows"]
        a, b = g["stats"][rows], r["stats"][rows]
        names = {"mean_U": slice(2, 5), "reynolds_stress": slice(5, 11), "mean_omega": slice(11, 12),
                 "mean_psi": slice(12, 12 + ns), "psi_variance": slice(12 + ns, 12 + 2 * ns)}
        extra["error_vs_fp64"] = {k: rel_l2(a[:, s], b[:, s]) for k, s in names.items() if s.stop > s.start}
        extra["fp64"] = dict(value=n * args.steps / (r["ms"] * 1e-3), ms_per_step=r["ms"] / args.steps,
                             particle_kernel_ms=r["k1_ms"] / max(r["k1_n"], 1))

    cpu = None
    if not args.no_cpu_baseline and rank == 0:
        cpu = cpu_baseline(cfg)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + "-" + args.precision, "particles": n, "elements": mesh.n_elems,
                   "stat_nodes": g["nsn"], "scalars": ns, "mode": params["mode"], "dt": params["dt"],
                   "sort_interval": opts["sort_interval"], "graph": opts["graph"],
                   "accumulation": "f64 node sums, f64 Eulerian fields and CG"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_particle_step", "kernel_ms": k1_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": nbytes, "bytes_per_particle": per_particle},
        "particle_kernel_updates_per_s": n / k1_avg_s,
        "counters": g["counters"],
        "cpu_baseline": cpu,
    }
    out.update(extra)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
