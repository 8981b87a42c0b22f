"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (graph replay, 256-thread blocks, sort every 10 steps), on what the
oracle can check one particle at a time.

Given the fields F^n, a particle's position, velocity, frequency, element and
velocity bin after one step depend on nothing but its own state and its
Wiener increments (the scalars also depend on the cell means, so they are not
compared). The oracle therefore advances a sample of particles, with the GPU's
F^n uploaded as frozen fields, and must reproduce the GPU's FP64 results bit
for bit. The total node weight must equal the total particle weight at any
size (R-11, mass conservation of the estimator).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_1006_0549_amd as P
    return P


def _sample_ids(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False))


def _check_sampled(oracle_mod, mesh, params, parts, F, after, ids, step_index=0, pressure=None, rtol=0.0):
    """Oracle: frozen fields F (and the mean pressure, whose gradient the
    step applies as the projection's correction), the sampled particles, one
    step (with the given step index in the random-number counter); compare,
    bit for bit unless rtol (relative to each quantity's scale) is given."""
    sub = {k: (v[..., ids] if isinstance(v, np.ndarray) and v.shape[-1] == len(parts["x"]) else v)
           for k, v in parts.items()}
    p0 = dict(params)
    p0["mode"] = 0
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, p0)
    o.fields_upload(oc, F)
    if pressure is not None:
        o.pressure_upload(oc, pressure)
    o.upload(oc, sub)
    o.init()
    o.set_step_index(step_index)
    o.step(1)
    r = o.download(oc, len(ids))
    g = {k: after[k][np.searchsorted(after["id"], r["id"])] for k in ("x", "y", "u", "v", "w", "omega", "elem", "bin", "id")}
    assert np.array_equal(g["id"], r["id"])
    assert np.array_equal(g["elem"], r["elem"]), np.nonzero(g["elem"] != r["elem"])[0][:5]
    for k in ("x", "y", "u", "v", "w", "omega"):
        bad = np.nonzero(np.abs(g[k] - r[k]) > rtol * np.abs(r[k]).max())[0]
        assert bad.size == 0, (k, bad[:5], g[k][bad[:5]], r[k][bad[:5]])
    assert np.array_equal(g["bin"], r["bin"])


def _by_id(d):
    order = np.argsort(d["id"])
    return {k: (v[..., order] if isinstance(v, np.ndarray) and v.shape[-1] == len(order) else v) for k, v in d.items()}


def test_channel_full_size_sampled_fp64(P, oracle_mod):
    cfg = W.config_channel()
    mesh, params, parts = cfg["mesh"], cfg["params"], cfg["particles"]
    n = len(parts["x"])
    _flush(f"[fullsize] channel {mesh.n_elems} triangles, {n} particles, FP64, graph replay")
    sim = P.Sim("fp64", "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.set_options(sort_interval=10, block_size=256, use_graph=True)
    sim.upload(cs, parts)
    sim.init()
    F = sim.fields(cs)
    sim.step(1)
    after = _by_id(sim.download(cs, n))
    S = sim.node_sums(cs)
    rows = np.unique(sim.case_info(cs)[1], return_index=True)[1]
    wsum = float(after["weight"].sum())
    assert abs(S[rows, 0].sum() - wsum) <= 1e-12 * wsum
    cnt = sim.counters(cs)
    assert cnt["nan"] == 0 and cnt["cg_fail"] == 0
    _flush("[fullsize] channel: oracle on 4096 sampled particles")
    _check_sampled(oracle_mod, mesh, params, parts, F, after, _sample_ids(n, 4096, 1))


def test_cavity_full_size_sampled_fp64(P, oracle_mod):
    """The lid-driven cavity at its full size (about 100k triangles refined at
    the walls, 100 particles per element, two scalars, sort every 10 steps,
    graph replay), FP64, after nine steps and the tenth with its sort: a
    sample of particles against the oracle with the GPU's fields and mean
    pressure frozen (elements and bins bit for bit, the state to 1e-14 of its
    scale), and the node weights adding up to the particle weight."""
    cfg = W.config_cavity()
    mesh, params, parts = cfg["mesh"], cfg["params"], cfg["particles"]
    n = len(parts["x"])
    _flush(f"[fullsize] cavity {mesh.n_elems} triangles, {n} particles, FP64, graph replay")
    sim = P.Sim("fp64", "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.set_options(sort_interval=10, block_size=256, use_graph=True)
    sim.upload(cs, parts)
    sim.init()
    sim.step(9)                  # the tenth step ends with a sort
    sim.synchronize()
    F = sim.fields(cs)
    Pm = sim.pressure(cs)
    before = _by_id(sim.download(cs, n))
    sim.step(1)
    after = _by_id(sim.download(cs, n))
    S = sim.node_sums(cs)
    rows = np.unique(sim.case_info(cs)[1], return_index=True)[1]
    wsum = float(after["weight"].sum())
    assert abs(S[rows, 0].sum() - wsum) <= 1e-12 * wsum
    cnt = sim.counters(cs)
    assert cnt["nan"] == 0 and cnt["cg_fail"] == 0, cnt
    # the sort at the end of the tenth step left the particles in (element, id) order
    d = sim.download(cs, n)
    key = d["elem"].astype(np.int64) * (1 << 32) + d["id"].astype(np.int64)
    assert np.all(np.diff(key) > 0)
    _flush("[fullsize] cavity: oracle on 4096 sampled particles")
    # the oracle recovers grad <P> from the uploaded <P> in its own summation
    # order, so the projection's correction may differ in the last bit
    _check_sampled(oracle_mod, mesh, params, before, F, after, _sample_ids(n, 4096, 3), step_index=9, pressure=Pm,
                   rtol=1e-14)


def test_batch32_full_size_sampled_fp64(P, oracle_mod):
    b = W.config_batched()
    cases = b["cases"]
    ntot = sum(len(c["particles"]["x"]) for c in cases)
    _flush(f"[fullsize] batch32: {len(cases)} cases, {ntot} particles, FP64, graph replay")
    sim = P.Sim("fp64", "cuda:0")
    ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in cases]
    sim.bind()
    sim.set_options(sort_interval=10, block_size=256, use_graph=True)
    for cs, c in zip(ids, cases):
        sim.upload(cs, c["particles"])
    sim.init()
    Fs = [sim.fields(cs) for cs in ids]
    sim.step(1)
    _flush("[fullsize] batch32: stepped; checking every case")
    for ci, (cs, c) in enumerate(zip(ids, cases)):
        n = len(c["particles"]["x"])
        after = _by_id(sim.download(cs, n))
        S = sim.node_sums(cs)
        rows = np.unique(sim.case_info(cs)[1], return_index=True)[1]
        wsum = float(after["weight"].sum())
        assert abs(S[rows, 0].sum() - wsum) <= 1e-12 * wsum, ci
        cnt = sim.counters(cs)
        assert cnt["nan"] == 0 and cnt["cg_fail"] == 0, (ci, cnt)
        _check_sampled(oracle_mod, c["mesh"], c["params"], c["particles"], Fs[ci], after, _sample_ids(n, 256, 100 + ci))
    _flush("[fullsize] batch32: all cases checked")


def test_batch32_projection_factor_matches_pcg(P):
    """The projection by the Cholesky factors (default; the tallest supernode
    trees and separators of more than 128 unknowns, which run with wide
    workgroups, occur only at these sizes) against the multigrid PCG of the
    same systems: after initialisation and two full FP64 steps of the 32-case
    batch, mean pressure and pressure gradients agree to far better than the
    PCG's own tolerance allows to matter."""
    b = W.config_batched()
    cases = b["cases"]
    _flush(f"[fullsize] batch32 projection: Cholesky sweeps against PCG, {len(cases)} cases")
    out = {}
    for method in ("direct", "pcg"):
        sim = P.Sim("fp64", "cuda:0")
        ids = [sim.add_case(c["mesh"], dict(c["params"], cg_rtol=1e-12), len(c["particles"]["x"])) for c in cases]
        sim.bind()
        sim.set_options(sort_interval=10, block_size=256, use_graph=True)
        sim.set_projection_solver(method)
        assert sim.projection_info()["method"] == method
        for cs, c in zip(ids, cases):
            sim.upload(cs, c["particles"])
        sim.init()
        sim.step(2)
        out[method] = [(sim.pressure(cs), sim.fields(cs)[:, 3:5], sim.counters(cs)) for cs in ids]
        _flush(f"[fullsize] batch32 projection: {method} done")
        del sim
    for ci, ((Pd, Gd, cd), (Pp, Gp, cp)) in enumerate(zip(out["direct"], out["pcg"])):
        assert cd["cg_iters_p"] == 0 and cp["cg_iters_p"] > 0 and cd["cg_fail"] == 0 and cp["cg_fail"] == 0
        sp = max(np.abs(Pp).max(), 1e-30)
        assert np.abs(Pd - Pp).max() <= 1e-6 * sp, (ci, np.abs(Pd - Pp).max() / sp)
        sg = max(np.abs(Gp).max(), 1e-30)
        assert np.abs(Gd - Gp).max() <= 1e-6 * sg, (ci, np.abs(Gd - Gp).max() / sg)


def test_batch32_sort_is_a_permutation_at_full_size(P):
    """The periodic sort at the benchmark size (452,500 elements, so the
    element-count scan spans 442 blocks): right after a sort every case's
    particles are ordered by element and still form the uploaded set, and a
    run that sorts every step follows the unsorted run (FP64, two steps)."""
    b = W.config_batched()
    cases = b["cases"]
    _flush(f"[fullsize] batch32 sort: {len(cases)} cases, FP64, sort every step against no sort")
    res = {}
    for si in (1, 0):
        sim = P.Sim("fp64", "cuda:0")
        ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in cases]
        sim.bind()
        sim.set_options(sort_interval=si, block_size=256, use_graph=True)
        for cs, c in zip(ids, cases):
            sim.upload(cs, c["particles"])
        sim.init()
        sim.step(2)
        if si == 1:
            sim.sort()
        res[si] = [sim.download(cs, len(c["particles"]["x"])) for cs, c in zip(ids, cases)]
        del sim
        _flush(f"[fullsize] batch32 sort: sort_interval={si} done")
    for ci, (a, b0) in enumerate(zip(res[1], res[0])):
        n = len(cases[ci]["particles"]["x"])
        assert np.array_equal(np.sort(a["id"]), np.arange(n)), ci
        assert np.all(np.diff(a["elem"]) >= 0), ci
        A, B = _by_id(a), _by_id(b0)
        # the node sums add in another order, so a particle on an element edge
        # may end in the neighbour; all others take the same path
        same = A["elem"] == B["elem"]
        assert same.mean() >= 1.0 - 1e-5, (ci, same.mean())
        for k in ("x", "y", "u", "v", "w", "omega"):
            assert np.allclose(A[k][same], B[k][same], rtol=1e-9, atol=1e-12), (ci, k)


def test_batch32_full_size_runs_twice_bitwise(P):
    """The benchmark's launch configuration (FP32, the 32-case batch, graph
    replay, block 256, sort every 5 steps, tail rows 256, adaptive PCG
    iterations) run twice from the same upload for 40 steps, sorts and
    changes of the unrolled iteration count included: the node sums,
    statistics and fields of every case are the same bits, and no element sum
    fell back to atomics."""
    b = W.config_batched()
    cases = b["cases"]
    _flush(f"[fullsize] batch32 run twice: {len(cases)} cases, FP32, graph replay, 40 steps each")
    out, iters = [], []
    for run in range(2):
        sim = P.Sim("fp32", "cuda:0")
        ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in cases]
        sim.bind()
        sim.set_options(sort_interval=5, block_size=256, use_graph=True)
        sim.set_solver(iterations=0, tail_rows=256)
        for cs, c in zip(ids, cases):
            sim.upload(cs, c["particles"])
        sim.init()
        it0 = sim.solver_info()[0]
        sim.step(40)
        iters.append((it0, sim.solver_info()[0]))
        out.append([(sim.node_sums(cs), sim.stats(cs), sim.fields(cs), sim.counters(cs)) for cs in ids])
        _flush(f"[fullsize] batch32 run twice: run {run} done, unrolled iterations {iters[-1]}")
        del sim
    assert iters[0] == iters[1] and iters[0][0] != iters[0][1], iters
    for ci, (a, b_) in enumerate(zip(*out)):
        assert a[3]["scatter_overflow"] == 0 and a[3]["nan"] == 0, (ci, a[3])
        for k in range(3):
            assert np.array_equal(a[k], b_[k]), (ci, k)


@pytest.mark.parametrize("precision,iterations,steps", [("fp32", 40, 3), ("fp64", 40, 3), ("fp32", 0, 24)],
                         ids=["fp32-fixed", "fp64-fixed", "fp32-adaptive"])
def test_batch32_full_size_batched_equals_sequential(P, precision, iterations, steps):
    """Each of the 32 cases stepped alone gives the bits it gets inside the
    batch (graph replay, sort every 5 steps): its sums, statistics and fields
    depend on its own particles and systems only. With a fixed count of
    row-parallel PCG iterations, and with the adaptive count over 24 steps
    (two readbacks): each system hands over to the one-workgroup completion
    at an iteration set from its own solves, so it takes the completion at
    the same iteration in both runs."""
    b = W.config_batched()
    cases = b["cases"]
    _flush(f"[fullsize] batch32 batched vs sequential: {len(cases)} cases, {precision}, iterations {iterations}, "
           f"{steps} steps")

    def run(sub):
        sim = P.Sim(precision, "cuda:0")
        ids = [sim.add_case(c["mesh"], c["params"], len(c["particles"]["x"])) for c in sub]
        sim.bind()
        sim.set_options(sort_interval=5, block_size=256, use_graph=True)
        sim.set_solver(iterations=iterations, tail_rows=256)
        for cs, c in zip(ids, sub):
            sim.upload(cs, c["particles"])
        sim.init()
        sim.step(steps)
        out = [(sim.node_sums(cs), sim.stats(cs), sim.fields(cs), sim.counters(cs)["scatter_overflow"]) for cs in ids]
        del sim
        return out

    together = run(cases)
    _flush("[fullsize] batch32 batched vs sequential: batch done")
    for ci, c in enumerate(cases):
        (alone,) = run([c])
        assert alone[3] == 0 and together[ci][3] == 0, ci
        for k in range(3):
            assert np.array_equal(alone[k], together[ci][k]), (ci, k)
    _flush("[fullsize] batch32 batched vs sequential: all cases equal")
