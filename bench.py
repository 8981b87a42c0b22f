"""Throughput of the particle advance on one MI355X.

One step = one pdfmc_step(1) over every case of the workload: particle kernel
(location by neighbour walk, P1 interpolation, GLM velocity / position /
frequency SDEs, IECM mixing, boundary conditions, scatter of the moments),
node statistics, cell means, Eulerian fields, elliptic-relaxation and
projection CG solves. Inputs are synthetic and resident in HBM before the
timed region starts.

    python bench.py [--steps K] [--warmup W] [--workload batch32|channel|cavity|small]
                    [--precision fp32|fp64] [--graph 0|1] [--sort-interval M]

Workloads: batch32 (default) is 32 independent channel and cavity cases
advanced together; channel and cavity are the single-case flows; small is the
450-triangle square. Prints one JSON line. Only one GPU is supported:
--gpus N > 1 exits.
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
    """Returns (name, list of cases, options); a case is dict(mesh, params, particles)."""
    import workloads as W
    if name == "batch32":
        b = W.config_batched()
        return b["name"], b["cases"], dict(sort_interval=10)
    if name == "channel":
        cfg = W.config_channel()
    elif name == "cavity":
        cfg = W.config_cavity()
    elif name == "small":
        cfg = W.config_small()
    else:
        raise SystemExit(f"unknown workload {name}")
    return cfg["name"], [cfg], dict(sort_interval=10)


PARTICLE_KERNEL_SOURCES = ["k_particle.hip", "pdfmc_dev.h", "pdfmc_math.h"]


def particle_kernel_hash():
    """SHA-1 of the particle kernel's sources: HBM counter readings are only
    valid for the kernel they were taken on."""
    import hashlib
    h = hashlib.sha1()
    for f in PARTICLE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1006_0549_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(workload_name, prec):
    """HBM bytes per particle-kernel launch from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes recorded in profiles/hbm_traffic.md (scaled by the
    readings of a plain copy of known size), or None when no row matches the
    workload, precision and current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    src = particle_kernel_hash()
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 9 and cells[0] == "k_particle_step" and cells[1] == workload_name and \
                cells[2] == prec and cells[3] == src:
            return float(cells[8])
    return None


def algorithmic_bytes(prec, cases, nsn):
    """Bytes the particle kernel must move per launch: every particle's state
    read and written once, the node fields (with the projection's gradient)
    read and node sums written once,
    element records and cell tables read/written once."""
    R = 4 if prec == "fp32" else 8
    total, npart = 0, 0
    for c, nn in zip(cases, nsn):
        ns = c["params"]["n_scalars"]
        n = len(c["particles"]["x"])
        ne = c["mesh"].n_elems
        per_particle = (7 * R + ns * R + 4 + 4 + 1) + (6 * R + ns * R + 4 + 1)
        per_node = 24 * R + 8 * (11 + 2 * ns)      # 22 fields + the velocity correction's 2
        per_elem = 8 * R + 12 + (8 * ns * R + 8 * (1 + ns) * 8 + 8 * 4 if ns else 0)
        total += n * per_particle + nn * per_node + ne * per_elem
        npart += n
    return total, total / max(npart, 1)


def run_gpu(cases, prec, steps, warmup, opts, repeats=1):
    import torch
    from paper_1006_0549_amd import Sim
    sim = Sim(prec, "cuda:0")
    ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in cases]
    ws = sim.bind()
    sim.set_options(sort_interval=opts.get("sort_interval", 0), block_size=opts.get("block_size", 256),
                    use_graph=opts.get("graph", False))
    sim.set_solver(iterations=opts.get("cg_iters", 0), tail_rows=opts.get("tail_rows", 64))
    sim.set_projection_solver(opts.get("projection", "direct"))
    for cs, c in zip(ids, cases):
        sim.upload(cs, c["particles"])
    sim.init()
    n = sum(len(c["particles"]["x"]) for c in cases)
    log(f"{prec}: {len(cases)} case(s), workspace {ws / 2**20:.1f} MiB, {n} particles; warmup {warmup} steps")
    sim.step(warmup)
    tuned = None
    if opts.get("autotune"):
        t0 = time.perf_counter()
        tuned = sim.autotune(steps_per_trial=4)
        log(f"{prec}: autotuner chose {tuned} in {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    # `repeats` timed windows of `steps` graph replays each; the median window counts
    windows = []
    for _ in range(max(1, repeats)):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(sim.stream)
        sim.step(steps)
        stop.record(sim.stream)
        torch.cuda.synchronize()
        windows.append((start.elapsed_time(stop), time.perf_counter() - t0))
    windows.sort()
    ms, wall = windows[len(windows) // 2]
    # particle-kernel duration: HIP events around each launch on the library's
    # stream (eager launches; the kernel is the same one the graph replays)
    kt = max(1, min(steps, 10))
    sim.timing(True)
    sim.step(kt)
    torch.cuda.synchronize()
    k1_ms, k1_n = sim.timing_read()
    sim.timing(False)
    log(f"{prec}: {steps} steps in {ms:.2f} ms (wall {wall * 1e3:.1f} ms); particle kernel "
        f"{k1_ms / max(k1_n, 1):.3f} ms/launch over {k1_n} launches")
    out = dict(ms=ms, k1_ms=k1_ms, k1_n=k1_n, n=n, stats=[], rows=[], nsn=[], counters={},
               windows_ms=[w[0] for w in windows],
               solver=sim.solver_info(), projection=sim.projection_info(), tuned=tuned)
    for cs in ids:
        nsn, sn = sim.case_info(cs)
        out["nsn"].append(nsn)
        out["rows"].append(np.unique(sn, return_index=True)[1])
        out["stats"].append(sim.stats(cs))
        for k, v in sim.counters(cs).items():
            out["counters"][k] = out["counters"].get(k, 0) + v
    del sim
    torch.cuda.synchronize()
    return out


def one_by_one(cases, prec, steps, warmup, opts):
    """The same cases advanced one at a time (one context each)."""
    total_ms, total_n = 0.0, 0
    for c in cases:
        r = run_gpu([c], prec, steps, warmup, opts)
        total_ms += r["ms"]
        total_n += r["n"] * steps
    return dict(value=total_n / (total_ms * 1e-3), ms_per_step=total_ms / steps)


def gpu_stats(cases, prec, steps, opts):
    """Node statistics of the cases after exactly `steps` steps from their
    initial state (one context, the benchmark's launch settings)."""
    import torch
    from paper_1006_0549_amd import Sim
    sim = Sim(prec, "cuda:0")
    ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in cases]
    sim.bind()
    sim.set_options(sort_interval=opts.get("sort_interval", 0), block_size=opts.get("block_size", 256),
                    use_graph=opts.get("graph", False))
    sim.set_solver(iterations=opts.get("cg_iters", 0), tail_rows=opts.get("tail_rows", 64))
    sim.set_projection_solver(opts.get("projection", "direct"))
    for cs, c in zip(ids, cases):
        sim.upload(cs, c["particles"])
    sim.init()
    sim.step(steps)
    torch.cuda.synchronize()
    out = [(sim.stats(cs), np.unique(sim.case_info(cs)[1], return_index=True)[1]) for cs in ids]
    del sim
    return out


def host_cpu():
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
    except OSError:
        pass
    name = info.get("model name", "unknown")
    return f"{name} (family {info.get('cpu family', '?')}, model {info.get('model', '?')}, " \
           f"stepping {info.get('stepping', '?')})"


def cpu_baseline(cases, opts, budget_s=30.0, max_steps=20):
    """The oracle leg. The oracle (single-threaded FP64 C, untuned) advances a
    bounded sample of the workload: the three smallest cases of a batch (the
    whole workload otherwise) for as many steps as fit in the budget, at most
    max_steps; that gives the CPU rate. The FP32 and FP64 GPU paths then
    advance the same sample for the same number of steps from the same
    initial state, and their node statistics are compared with the oracle's:
    relative L2 error per group of statistics and the fraction of (node,
    statistic) pairs inside three standard errors (oracle/band.py)."""
    import oracle
    from oracle import band
    sample = sorted(cases, key=lambda c: len(c["particles"]["x"]))[:3]
    n = sum(len(c["particles"]["x"]) for c in sample)
    o = oracle.Oracle()
    ocs = [o.add_case(c["mesh"], c["params"]) for c in sample]
    for oc, c in zip(ocs, sample):
        o.upload(oc, c["particles"])
    t0 = time.perf_counter()
    o.init()
    log(f"oracle init {time.perf_counter() - t0:.1f} s")
    done, t = 0, 0.0
    while t < budget_s and done < max_steps:
        t1 = time.perf_counter()
        o.step(1)
        t += time.perf_counter() - t1
        done += 1
        log(f"oracle step {done}: {t:.1f} s")
    ref = [(o.stats(oc), o.node_sums(oc)) for oc in ocs]
    what = "the three smallest cases of the batch" if len(cases) > 1 else "the workload"
    names = ", ".join(f"{c['mesh'].name} ({len(c['particles']['x'])} particles, {c['params']['n_scalars']} scalars)"
                      for c in sample)
    cpu = dict(value=n * done / t, unit="particle-updates/s", cores=1, kind="oracle", host_cpu=host_cpu(),
               host_threads=os.cpu_count(),
               sample=f"{done} full steps of {what}: {names}; single-threaded FP64 C, timed after initialisation")
    prec = {}
    for p_ in ("fp32", "fp64"):
        g = gpu_stats(sample, p_, done, dict(opts, autotune=False))
        groups, fr = {}, {}
        for c, (gst, rows), (rst, sums) in zip(sample, g, ref):
            ns = c["params"]["n_scalars"]
            for k, cols in band.columns(ns).items():
                if cols:
                    groups.setdefault(k, []).append((gst[rows][:, cols].ravel(), rst[rows][:, cols].ravel()))
            for k, v in band.fractions(gst, rst, sums, ns, rows=rows).items():
                fr.setdefault(k, []).append((v["fraction"], len(rows) * len(band.columns(ns)[k])))
        prec[p_] = dict(
            rel_l2={k: rel_l2(np.concatenate([a for a, _ in v]), np.concatenate([b for _, b in v]))
                    for k, v in groups.items()},
            in_3_sigma={k: float(sum(f * w for f, w in v) / sum(w for _, w in v)) for k, v in fr.items()})
        log(f"{p_} against the oracle after {done} steps: {prec[p_]}")
    return cpu, dict(steps=done, sample=names, **prec)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def error_vs_fp64(cases, g, r):
    """Relative L2 error of each statistic over all statistics nodes of all cases."""
    groups = {"mean_U": [], "reynolds_stress": [], "mean_omega": [], "mean_psi": [], "psi_variance": []}
    refs = {k: [] for k in groups}
    for c, a, b, rows in zip(cases, g["stats"], r["stats"], g["rows"]):
        ns = c["params"]["n_scalars"]
        sl = {"mean_U": slice(2, 5), "reynolds_stress": slice(5, 11), "mean_omega": slice(11, 12),
              "mean_psi": slice(12, 12 + ns), "psi_variance": slice(12 + ns, 12 + 2 * ns)}
        for k, s in sl.items():
            if s.stop > s.start:
                groups[k].append(a[rows, s].reshape(-1))
                refs[k].append(b[rows, s].reshape(-1))
    return {k: rel_l2(np.concatenate(groups[k]), np.concatenate(refs[k])) for k in groups if groups[k]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch32")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--sort-interval", type=int, default=None)
    ap.add_argument("--block-size", type=int, default=256)
    ap.add_argument("--repeats", type=int, default=3, help="timed windows of --steps steps; the median is reported")
    ap.add_argument("--cg-iters", type=int, default=0, help="row-parallel CG iterations per step (0: adaptive)")
    ap.add_argument("--tail-rows", type=int, default=64, help="multigrid levels at most this size run in one workgroup")
    ap.add_argument("--projection", default="direct", choices=["direct", "pcg"],
                    help="projection solve: Cholesky factor sweeps or multigrid PCG")
    ap.add_argument("--autotune", type=int, default=None,
                    help="run the autotuner before the timed steps (default: on for batch32)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied by a plain device copy before the workload (reference kernel for HBM counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-one-by-one", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: only one GPU is measured (the particle advance is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration > 0:
        import torch
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read and written, 3 times")
        del src, dst
    t0 = time.perf_counter()
    name, cases, opts = workload(args.workload)
    if args.sort_interval is not None:
        opts["sort_interval"] = args.sort_interval
    opts["graph"] = bool(args.graph)
    opts["block_size"] = args.block_size
    opts["cg_iters"] = args.cg_iters
    opts["tail_rows"] = args.tail_rows
    opts["projection"] = args.projection
    opts["autotune"] = bool(args.autotune if args.autotune is not None else args.workload == "batch32")
    n = sum(len(c["particles"]["x"]) for c in cases)
    ne = sum(c["mesh"].n_elems for c in cases)
    scal = [c["params"]["n_scalars"] for c in cases]
    log(f"workload {name}: {len(cases)} case(s), {ne} triangles, {n} particles "
        f"(inputs built in {time.perf_counter() - t0:.1f} s)")

    g = run_gpu(cases, args.precision, args.steps, args.warmup, opts, repeats=args.repeats)
    if g["tuned"]:
        # the other legs run with the settings the autotuner chose
        opts.update(block_size=g["tuned"]["block_size"], sort_interval=g["tuned"]["sort_interval"],
                    tail_rows=g["tuned"]["tail_rows"], autotune=False)
    ms_per_step = g["ms"] / args.steps
    value = n * args.steps / (g["ms"] * 1e-3)
    k1_avg_s = g["k1_ms"] / max(g["k1_n"], 1) * 1e-3
    nbytes, per_particle = algorithmic_bytes(args.precision, cases, g["nsn"])
    achieved = nbytes / k1_avg_s / 1e9

    extra = {}
    if args.precision == "fp32" and not args.no_fp64_reference:
        # the same number of steps as the FP32 run (its autotuner trials included)
        more = g["tuned"]["steps"] if g["tuned"] else 0
        r = run_gpu(cases, "fp64", args.steps, args.warmup + more, opts, repeats=args.repeats)
        extra["error_vs_fp64"] = error_vs_fp64(cases, g, r)
        # the statistical noise of the same comparison: FP64 against FP64 on
        # another random-number stream (the statistics are one-step particle
        # estimates, so two runs differ by their sampling noise)
        alt = [dict(c, params=dict(c["params"], stream=int(c["params"]["stream"]) + 977)) for c in cases]
        r2 = run_gpu(alt, "fp64", args.steps, args.warmup + more, opts, repeats=1)
        noise = error_vs_fp64(cases, r2, r)
        extra["fp64_vs_fp64_other_stream"] = noise
        extra["error_over_noise"] = {k: extra["error_vs_fp64"][k] / max(v, 1e-300) for k, v in noise.items()
                                     if k in extra["error_vs_fp64"]}
        extra["fp64"] = dict(value=n * args.steps / (r["ms"] * 1e-3), ms_per_step=r["ms"] / args.steps,
                             particle_kernel_ms=r["k1_ms"] / max(r["k1_n"], 1),
                             fp32_speedup=r["ms"] / g["ms"])
    if len(cases) > 1 and not args.no_one_by_one:
        s = one_by_one(cases, args.precision, 5, 2, opts)
        extra["one_by_one"] = dict(value=s["value"], ms_per_step=s["ms_per_step"],
                                   batched_speedup=value / s["value"], steps=5)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, extra["precision_vs_oracle"] = cpu_baseline(cases, opts)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "timed_windows_ms": g["windows_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{name}-{args.precision}", "cases": len(cases), "particles": n,
                   "elements": ne, "stat_nodes": int(sum(g["nsn"])), "scalars": scal if len(scal) > 1 else scal[0],
                   "sort_interval": opts["sort_interval"], "graph": opts["graph"],
                   "block_size": opts["block_size"], "tail_rows": opts["tail_rows"],
                   "cg_row_parallel_iterations": g["solver"][0], "cg_row_parallel_levels": g["solver"][1],
                   "projection": g["projection"]["method"],
                   "projection_factor_values": g["projection"]["factor_values"],
                   "autotuned": g["tuned"],
                   "accumulation": "f64 node sums, f64 Eulerian fields and CG"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, args.precision),
                     "kernel_source": particle_kernel_hash(),
                     "kernel": "k_particle_step", "kernel_ms": k1_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": nbytes, "bytes_per_particle": per_particle},
        "particle_kernel_updates_per_s": n / k1_avg_s,
        "counters": g["counters"],
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
