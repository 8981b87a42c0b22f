"""GPU parity of the HIP particle advance against the FP64 CPU oracle, through
the C ABI (include/pdfmc.h).

Bar (FP64 path): element ids, velocity bins and the full particle state are
bit-identical after a step from identical state; node sums agree to 1e-13 of
sum |w N Q| (the GPU sums in its own fixed order, not the oracle's); statistics to
1e-12 relative to their scale for one step and 1e-9 over a 100-step run with
live fields. Cases span several tiles and a ragged last tile, walls, periodic
edges, sources, 1 and 2 scalars, 8 velocity bins.
"""
import os

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


def _pair(P, oracle_mod, mesh, params, parts, precision="fp64", fields=None, options=None, solver=None):
    n = len(parts["x"])
    sim = P.Sim(precision, "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    if options:
        sim.set_options(**options)
    if solver:
        solver = dict(solver)
        proj = solver.pop("projection", None)
        if solver:
            sim.set_solver(**solver)
        if proj:
            sim.set_projection_solver(proj)
    if fields is not None:
        sim.fields_upload(cs, fields)
    sim.upload(cs, parts)
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, params)
    if fields is not None:
        o.fields_upload(oc, fields)
    o.upload(oc, parts)
    return sim, cs, o, oc


def _stat_rows(sim, cs):
    _, sn = sim.case_info(cs)
    return np.unique(sn, return_index=True)[1]


def _scale(st, ns):
    """scale of each statistic: |<Q>| for means, and for central moments the
    raw second moments sqrt(<Q^2><Q'^2>) (the size of what cancels)"""
    sc = np.abs(st).copy()
    raw = st[:, 5:8] + st[:, 2:5] ** 2                  # <U_i^2>
    for c, i in ((5, 0), (6, 1), (7, 2)):
        sc[:, c] = raw[:, i]
    for c, (i, j) in {8: (0, 1), 9: (0, 2), 10: (1, 2)}.items():
        sc[:, c] = np.sqrt(raw[:, i] * raw[:, j])
    for a in range(ns):
        sc[:, 12 + ns + a] = st[:, 12 + ns + a] + st[:, 12 + a] ** 2
    return np.maximum(sc, 1e-300)


def _assert_state_equal(g, r, keys=("x", "y", "u", "v", "w", "omega")):
    assert np.array_equal(g["elem"], r["elem"]), np.nonzero(g["elem"] != r["elem"])[0][:10]
    for k in keys:
        bad = np.nonzero(g[k] != r[k])[0]
        assert bad.size == 0, (k, bad[:5], g[k][bad[:5]], r[k][bad[:5]])
    if r["psi"].size:
        # mixing uses cell means, i.e. FP64 sums in another order than the oracle's:
        # |delta psi| <= (dt/t_m) |delta mean| ~ a few ulp of the scalar scale
        d = np.abs(g["psi"] - r["psi"])
        assert d.max() <= 1e-14 * max(1.0, np.abs(r["psi"]).max()), d.max()


def test_gaussians_bitwise_fp64(P, oracle_mod):
    sim = P.Sim("fp64", "cuda:0")
    ids = np.arange(0, 20000, dtype=np.uint32) * 7919
    g = sim.draw_gaussians(10060549, 17, 3, ids)
    r = np.array([oracle_mod.gauss6(10060549, int(i), 17, 3) for i in ids])
    assert np.array_equal(g, r), np.max(np.abs(g - r))


def test_gaussians_fp32_follow_fp64(P, oracle_mod):
    sim = P.Sim("fp32", "cuda:0")
    ids = np.arange(50000, dtype=np.uint32)
    g = sim.draw_gaussians(10060549, 5, 1, ids).astype(np.float64)
    for j in range(6):
        assert abs(g[:, j].mean()) < 4.5 / np.sqrt(len(ids))
        assert abs(g[:, j].var() - 1.0) < 4.5 * np.sqrt(2.0 / len(ids))
    r = np.array([oracle_mod.gauss6(10060549, int(i), 5, 1) for i in ids[:3000]])
    d = np.abs(g[:3000] - r)
    assert np.median(d) < 1e-5 and np.quantile(d, 0.99) < 1e-3


def _frozen_case(ns=1, nb=8, n=16, ppe=33, seed=5):
    mesh = W.unit_square(n, 0.2, periodic_x=True, periodic_y=False, lid=(0.5, 0.0, 0.0), seed_key=(5, 0, 0))
    rng = np.random.default_rng(seed)
    F = W.frozen_fields(mesh, C0=2.1, omega=1.3, k=0.02, dpdx=(-1.0, 0.2))
    F[:, 0:3] = rng.normal(0, 0.05, (mesh.n_nodes, 3))
    F[:, 5:11] = rng.normal(0, 0.5, (mesh.n_nodes, 6))
    F[:, 11:14] = rng.normal(0, 1.0, (mesh.n_nodes, 3))
    F[:, 15:17] = rng.normal(0, 0.3, (mesh.n_nodes, 2))
    F[:, 21] = rng.normal(0.7, 0.1, mesh.n_nodes)
    # periodic images must carry equal fields: copy left column onto the right
    right = np.nonzero(mesh.xy[:, 0] == 1.0)[0]
    for r_ in right:
        l_ = np.nonzero((mesh.xy[:, 0] == 0.0) & (mesh.xy[:, 1] == mesh.xy[r_, 1]))[0][0]
        F[r_] = F[l_]
    params = W.default_params(mode=0, dt=2e-3, nu=2e-3, n_scalars=ns, n_bins=nb,
                              src=[(0.3, 0.7, 0.08, 1.0), (0.6, 0.2, 0.1, 0.5), (0.8, 0.8, 0.1, 0.0),
                                   (0.15, 0.3, 0.1, 0.7)][:ns])
    parts = W.init_particles(mesh, ppe, ns, rng, u_std=0.4,
                             psi_disks=[(0.5, 0.5, 0.25, 1.0), (0.2, 0.8, 0.3, 2.0), (0.7, 0.3, 0.2, 0.0),
                                        (0.4, 0.6, 0.3, 1.5)][:ns])
    return mesh, params, parts, F


@pytest.mark.parametrize("ns,nb", [(1, 8), (2, 8), (0, 1), (1, 1)])
def test_one_step_frozen_bitwise(P, oracle_mod, ns, nb):
    mesh, params, parts, F = _frozen_case(ns, nb)
    n = len(parts["x"])
    _flush(f"[one_step_frozen] ns={ns} nb={nb} particles={n} tiles={(n + 255) // 256}")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, fields=F)
    sim.init(); o.init()
    # bins and cell means of the initial state
    assert np.array_equal(sim.download(cs, n)["bin"], o.download(oc, n)["bin"])
    if ns > 0:   # cells exist only where there are scalars to mix
        gm, gc = sim.cell_means(cs)
        rm, rc = o.cell_means(oc)
        assert np.array_equal(gc, rc)
        np.testing.assert_allclose(gm, rm, rtol=1e-13, atol=1e-15)
    for step in range(3):
        sim.step(1); o.step(1)
        g, r = sim.download(cs, n), o.download(oc, n)
        _assert_state_equal(g, r)
        assert np.array_equal(g["bin"], r["bin"])
        gs, rs = sim.node_sums(cs), o.node_sums(oc)
        # |delta| <= 1e-13 of the largest node sum of that moment
        tol = 1e-13 * np.abs(rs).max(0) + 1e-300
        assert np.all(np.abs(gs - rs) <= np.maximum(tol, 1e-13 * np.abs(rs))), np.max(np.abs(gs - rs))
        gst, rst = sim.stats(cs), o.stats(oc)
        rows = _stat_rows(sim, cs)
        d = np.abs(gst - rst)[rows] / _scale(rst, ns)[rows]
        assert d.max() <= 1e-12, (step, d.max(), np.unravel_index(np.argmax(d), d.shape))
    gc_, rc_ = sim.counters(cs), o.counters(oc)
    for k in ("walk_fallback", "reflect", "periodic", "omega_flip", "nan", "walk_steps"):
        assert gc_[k] == rc_[k], (k, gc_[k], rc_[k])
    assert rc_["reflect"] > 0 and rc_["periodic"] > 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_walk_caps_follow_the_oracle(P, oracle_mod, precision):
    """Particles set from the host so that both caps of the walk are reached
    in one step, on a coarse mesh (three element rows): five with a
    wall-normal velocity that crosses the unit square twelve times (the
    eighth reflection ends the walk, R-14), five with a streamwise velocity
    that crosses about 180 elements through the periodic edges (the 64-step
    cap, R-13); both end in the fallback. In FP64 the
    state and the counters equal the oracle's bit for bit; in FP32 (best
    visited element as the fallback) the counters show both caps and every
    particle keeps a valid element."""
    mesh = W.unit_square(4, 0.2, periodic_x=True, periodic_y=False, seed_key=(9, 0, 0))
    params = W.default_params(mode=0, dt=1e-3, nu=1e-4, n_scalars=0)
    parts = W.init_particles(mesh, 12, 0, W.rng_for(9, 0, 1), u_std=0.1)
    parts["v"][:5] = 12000.0
    parts["u"][5:10] = 30000.0
    n = len(parts["x"])
    F = W.frozen_fields(mesh, C0=2.1, omega=1.0, k=0.01)
    _flush(f"[walk_caps] {precision}: {n} particles, ten at extreme velocities, one step")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, precision=precision, fields=F)
    sim.init(); o.init()
    sim.step(1); o.step(1)
    gc_, rc_ = sim.counters(cs), o.counters(oc)
    assert rc_["walk_fallback"] >= 10 and rc_["reflect"] >= 5 * 8, rc_
    assert gc_["walk_fallback"] >= 10 and gc_["reflect"] >= 5 * 8, gc_
    g, r = sim.download(cs, n), o.download(oc, n)
    assert g["elem"].min() >= 0 and g["elem"].max() < mesh.n_elems
    if precision == "fp64":
        _assert_state_equal(g, r)
        for k in ("walk_fallback", "reflect", "periodic", "walk_steps"):
            assert gc_[k] == rc_[k], (k, gc_[k], rc_[k])
    else:
        # the other particles take the same elements as in FP64 (up to rounding on an edge)
        assert (g["elem"][10:] == r["elem"][10:]).mean() > 0.97


def test_frozen_table_overflow(P, oracle_mod):
    """Two particles per element: a workgroup of 256 particles meets about
    128 elements, more than its 32 regular record slots, so the rest take
    records from the pool, and once the pool is exhausted the element sums go
    to the FP64 overflow sums (counted as scatter overflow). The FP64 state,
    node sums, cell means and statistics still match the oracle after each
    step."""
    ns, nb = 2, 8
    mesh, params, parts, F = _frozen_case(ns, nb, ppe=2)
    n = len(parts["x"])
    _flush(f"[frozen_table_overflow] ns={ns} nb={nb} particles={n} tiles={(n + 255) // 256}")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, fields=F)
    sim.init(); o.init()
    gm, gc = sim.cell_means(cs)
    rm, rc = o.cell_means(oc)
    assert np.array_equal(gc, rc)
    np.testing.assert_allclose(gm, rm, rtol=1e-13, atol=1e-15)
    for step in range(3):
        sim.step(1); o.step(1)
        g, r = sim.download(cs, n), o.download(oc, n)
        _assert_state_equal(g, r)
        assert np.array_equal(g["bin"], r["bin"])
        gs, rs = sim.node_sums(cs), o.node_sums(oc)
        tol = 1e-13 * np.abs(rs).max(0) + 1e-300
        assert np.all(np.abs(gs - rs) <= np.maximum(tol, 1e-13 * np.abs(rs))), np.max(np.abs(gs - rs))
        gm, gc = sim.cell_means(cs)
        rm, rc = o.cell_means(oc)
        assert np.array_equal(gc, rc)
        np.testing.assert_allclose(gm, rm, rtol=1e-12, atol=1e-14)
        gst, rst = sim.stats(cs), o.stats(oc)
        rows = _stat_rows(sim, cs)
        # With about a dozen particles per node a mean of U or psi can be a
        # near-cancelling sum: the summation order (atomics here, particle
        # order in the oracle) moves it by about n eps sum|w Q| / W, which is
        # at most n eps <Q^2>^(1/2). So the means are scaled by their RMS
        # here, the size of what is summed, as the central moments already are.
        sc = _scale(rst, ns)
        sc[:, 2:5] = np.maximum(sc[:, 2:5], np.sqrt(np.maximum(rst[:, 5:8] + rst[:, 2:5] ** 2, 0.0)))
        for a in range(ns):
            sc[:, 12 + a] = np.maximum(sc[:, 12 + a], np.sqrt(np.maximum(rst[:, 12 + ns + a] + rst[:, 12 + a] ** 2, 0.0)))
        d = np.abs(gst - rst)[rows] / sc[rows]
        assert d.max() <= 1e-12, (step, d.max(), np.unravel_index(np.argmax(d), d.shape))
    assert sim.counters(cs)["scatter_overflow"] > 0


@pytest.mark.parametrize("reaction,ns,k", [(1, 2, (3.0, 0.7, 0.0, 0.0)), (2, 3, (4.0, 0.0, 0.0, 0.0)),
                                            (2, 4, (2.5, 0.0, 0.0, 0.0))])
def test_reaction_frozen_bitwise(P, oracle_mod, reaction, ns, k):
    """Reactive scalars (R-35): the FP64 particle state after each of three
    frozen-field steps equals the oracle's (scalars to the cell-mean rounding
    bound), with sources, walls, periodic edges and 8 velocity bins."""
    mesh, params, parts, F = _frozen_case(ns, 8)
    params.update(reaction=reaction, k_react=k)
    n = len(parts["x"])
    _flush(f"[reaction_frozen] reaction={reaction} ns={ns} particles={n}")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, fields=F)
    sim.init(); o.init()
    p0 = sim.download(cs, n)["psi"].copy()
    for step in range(3):
        sim.step(1); o.step(1)
        g, r = sim.download(cs, n), o.download(oc, n)
        _assert_state_equal(g, r)
        gst, rst = sim.stats(cs), o.stats(oc)
        rows = _stat_rows(sim, cs)
        d = np.abs(gst - rst)[rows] / _scale(rst, ns)[rows]
        assert d.max() <= 1e-12, (step, d.max())
    # the source acted: compositions differ from a passive run of the same case
    passive = dict(params, reaction=0)
    sim2, cs2, _, _ = _pair(P, oracle_mod, mesh, passive, parts, fields=F)
    sim2.init(); sim2.step(3)
    assert np.abs(sim2.download(cs2, n)["psi"] - g["psi"]).max() > 1e-4
    assert not np.array_equal(p0, g["psi"])


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_reaction_uniform_recursion(P, precision, rtol):
    """A uniform composition never mixes, so under A + B -> P every particle
    follows a_{n+1} = a_n - dt k a_n^2 (computed here in FP64); in FP32 to the
    rounding of the FP32 recursion."""
    mesh, params, parts, F = _frozen_case(3, 8)
    k, a0, steps = 5.0, 0.8, 25
    params.update(reaction=2, k_react=(k, 0.0, 0.0, 0.0), src=[])
    n = len(parts["x"])
    parts["psi"] = np.stack([np.full(n, a0), np.full(n, a0), np.zeros(n)])
    _flush(f"[reaction_uniform] {precision} particles={n} steps={steps}")
    sim = P.Sim(precision, "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.fields_upload(cs, F)
    sim.upload(cs, parts)
    sim.init()
    sim.step(steps)
    psi = sim.download(cs, n)["psi"]
    a = a0
    for _ in range(steps):
        a = a - params["dt"] * k * a * a
    np.testing.assert_allclose(psi[0], a, rtol=rtol, atol=0)
    np.testing.assert_allclose(psi[1], a, rtol=rtol, atol=0)
    np.testing.assert_allclose(psi[2], a0 - a, rtol=50 * rtol, atol=1e-5 if precision == "fp32" else 1e-15)


def test_small_config_100_steps(P, oracle_mod):
    cfg = W.config_small()
    parts = cfg["particles"]
    n = len(parts["x"])
    _flush(f"[small_config] {cfg['name']} particles={n} steps=100")
    sim, cs, o, oc = _pair(P, oracle_mod, cfg["mesh"], cfg["params"], parts)
    sim.init(); o.init()
    sim.step(100); o.step(100)
    g, r = sim.download(cs, n), o.download(oc, n)
    same = g["elem"] == r["elem"]
    assert same.mean() > 0.999, same.mean()
    gst, rst = sim.stats(cs), o.stats(oc)
    rows = _stat_rows(sim, cs)
    d = (np.abs(gst - rst)[rows] / _scale(rst, 1)[rows])
    assert d.max() <= 1e-9, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    gF, rF = sim.fields(cs), o.fields(oc)
    dF = np.abs(gF - rF)[rows] / np.maximum(np.abs(rF[rows]), 1e-6)
    assert dF.max() <= 1e-8, dF.max()


def _small_channel(ppe=20, ns=1, rtol=1e-13):
    mesh = W.channel(n_half=10, nx=24, seed_key=(1, 1, 0))
    params = W.default_params(mode=2, dt=5e-4, nu=1.0 / 1080.0, n_scalars=ns, dpdx=(-1.0, 0.0),
                              src=[(1.0, 0.5, 0.1, 1.0), (3.0, 1.5, 0.1, 1.0)][:ns], cg_rtol=rtol, cg_maxit=20000,
                              stream=1)
    parts = W.init_particles(mesh, ppe, ns, W.rng_for(1, 1, 1), u_std=1.0)
    return mesh, params, parts


@pytest.mark.parametrize("solver", [None, dict(projection="pcg"), dict(iterations=0, tail_rows=64, projection="pcg"),
                                    dict(iterations=2, tail_rows=64), dict(iterations=40, tail_rows=0, projection="pcg")],
                         ids=["default", "pcgprojection", "rowparallel", "finisher", "allrowparallel"])
def test_elliptic_relaxation_and_projection(P, oracle_mod, solver):
    """Relaxation and projection fields against the oracle. The projection
    runs on the Cholesky factor (default) or on the multigrid PCG; the solver
    options move the multigrid levels between the row-parallel phase kernels
    and the one-workgroup tail, and force the one-workgroup completion of
    systems that need more iterations than the phases ran."""
    mesh, params, parts = _small_channel()
    n = len(parts["x"])
    _flush(f"[er] channel {mesh.n_elems} triangles, {n} particles, mode 2, solver {solver}")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, solver=solver)
    if solver and solver.get("tail_rows", 1024) < 100:
        it, big = sim.solver_info()
        assert big >= 1
    sim.init(); o.init()
    rows = _stat_rows(sim, cs)
    gF, rF = sim.fields(cs)[rows], o.fields(oc)[rows]
    # field scales: per slot, the largest magnitude over the nodes
    sc = np.maximum(np.abs(rF).max(0), 1e-12)
    d = np.abs(gF - rF) / sc
    assert d.max() <= 1e-9, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    for step in range(4):
        sim.step(1); o.step(1)
    g, r = sim.download(cs, n), o.download(oc, n)
    assert (g["elem"] == r["elem"]).mean() > 0.999
    gst, rst = sim.stats(cs)[rows], o.stats(oc)[rows]
    d = np.abs(gst - rst) / _scale(rst, 1)
    assert d.max() <= 1e-8, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    gF, rF = sim.fields(cs)[rows], o.fields(oc)[rows]
    sc = np.maximum(np.abs(rF).max(0), 1e-12)
    d = np.abs(gF - rF) / sc
    assert d.max() <= 1e-7, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    gc_ = sim.counters(cs)
    assert gc_["cg_fail"] == 0 and gc_["cg_iters_er"] > 0
    direct = sim.projection_info()["method"] == "direct"
    assert direct == (not solver or solver.get("projection", "direct") == "direct")
    assert (gc_["cg_iters_p"] == 0) if direct else (gc_["cg_iters_p"] > 0)


def _fp32_cases():
    cfg = W.config_small()
    ch = W.channel(n_half=8, nx=20, seed_key=(1, 3, 0))
    chp = W.default_params(mode=2, dt=5e-4, nu=1.0 / 1080.0, n_scalars=1, dpdx=(-1.0, 0.0),
                           src=[(3.0, 1.0, 0.2, 1.0)], stream=5)
    chparts = W.init_particles(ch, 60, 1, W.rng_for(1, 3, 1), u_std=1.0)
    return [("square-mode1", cfg["mesh"], cfg["params"], cfg["particles"], 100),
            ("channel-mode2", ch, chp, chparts, 60)]


@pytest.mark.parametrize("case", range(2), ids=[c[0] for c in _fp32_cases()])
def test_fp32_statistical_band(P, oracle_mod, case):
    """The FP32 path against the FP64 oracle over a run: at every statistics
    node, every statistic (<U_i>, <u_i u_j>, <omega>, <psi>, <psi'^2>) within
    three standard errors of the oracle's, the standard error taken from the
    node's effective sample size W^2 / sum (w lambda)^2 (oracle/band.py), at
    99% of the (node, statistic) pairs or more; mode 1 on the small square and
    the full model (relaxation and projection) on a small channel."""
    from oracle import band
    name, mesh, params, parts, steps = _fp32_cases()[case]
    n = len(parts["x"])
    ns = params["n_scalars"]
    _flush(f"[fp32-band] {name}: {n} particles, {steps} steps, FP32 against the FP64 oracle")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, precision="fp32")
    sim.init(); o.init()
    sim.step(steps); o.step(steps)
    rows = _stat_rows(sim, cs)
    gst, rst, sums = sim.stats(cs), o.stats(oc), o.node_sums(oc)
    fr = band.fractions(gst, rst, sums, ns, rows=rows)
    _flush(f"[fp32-band] {name}: " + ", ".join(f"{k} {v['fraction']:.4f} (median {v['median_sigma']:.2g} sigma)"
                                              for k, v in fr.items()))
    for k, v in fr.items():
        assert v["fraction"] >= 0.99, (k, v)
        # the same Wiener path: typically far inside the band
        assert v["median_sigma"] < 0.5, (k, v)
    # the particles themselves stay close to the FP64 ones
    g, r = sim.download(cs, n), o.download(oc, n)
    assert (g["elem"] == r["elem"]).mean() > 0.99
    du = np.abs(g["u"] - r["u"]) / np.std(r["u"])
    assert np.median(du) < 1e-3, np.median(du)


def _run(P, mesh, params, parts, steps, precision="fp64", **opt):
    n = len(parts["x"])
    sim = P.Sim(precision, "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    if opt:
        sim.set_options(**opt)
    sim.upload(cs, parts)
    sim.init()
    sim.step(steps)
    return sim, cs


def _by_id(d):
    order = np.argsort(d["id"])
    return {k: (v[..., order] if isinstance(v, np.ndarray) and v.shape[-1] == len(order) else v) for k, v in d.items()}


@pytest.mark.parametrize("opts", [dict(sort_interval=3), dict(use_graph=True), dict(sort_interval=4, use_graph=True),
                                  dict(block_size=64)])
def test_sort_graph_block_invariance(P, opts):
    cfg = W.config_small()
    parts = cfg["particles"]
    n = len(parts["x"])
    _flush(f"[invariance] options {opts}")
    a, ca = _run(P, cfg["mesh"], cfg["params"], parts, 20)
    b, cb = _run(P, cfg["mesh"], cfg["params"], parts, 20, **opts)
    A, B = _by_id(a.download(ca, n)), _by_id(b.download(cb, n))
    assert np.array_equal(A["id"], np.arange(n))
    assert np.array_equal(B["id"], np.arange(n))
    assert (A["elem"] == B["elem"]).mean() > 0.999
    for k in ("x", "y", "u", "v", "w", "omega"):
        assert np.max(np.abs(A[k] - B[k])) <= 1e-10, k
    sa, sb = a.stats(ca), b.stats(cb)
    assert np.max(np.abs(sa - sb) / np.maximum(np.abs(sa), 1e-3)) <= 1e-9


def test_batched_equals_sequential(P):
    cfg = W.config_small()
    mesh2, params2, parts2 = _small_channel(ppe=10, ns=2, rtol=1e-12)
    _flush("[batched] two cases in one context against one context each")
    sim = P.Sim("fp64", "cuda:0")
    c1 = sim.add_case(cfg["mesh"], cfg["params"], len(cfg["particles"]["x"]))
    c2 = sim.add_case(mesh2, params2, len(parts2["x"]))
    sim.bind()
    sim.upload(c1, cfg["particles"]); sim.upload(c2, parts2)
    sim.init(); sim.step(5)
    a, ca = _run(P, cfg["mesh"], cfg["params"], cfg["particles"], 5)
    b, cb = _run(P, mesh2, params2, parts2, 5)
    for (s_b, c_b), (s_s, c_s), parts in (((sim, c1), (a, ca), cfg["particles"]), ((sim, c2), (b, cb), parts2)):
        n = len(parts["x"])
        G, S = s_b.download(c_b, n), s_s.download(c_s, n)
        assert (G["elem"] == S["elem"]).mean() > 0.999
        assert np.max(np.abs(G["u"] - S["u"])) <= 1e-10
        sb, ss = s_b.stats(c_b), s_s.stats(c_s)
        assert np.max(np.abs(sb - ss) / np.maximum(np.abs(ss), 1e-3)) <= 1e-8


def test_autotune_settings_and_invariance(P):
    """The autotuner picks settings from its candidate sets, and the steps it
    takes are ordinary steps. With frozen fields and no scalars a particle's
    path depends on nothing but its own state, so the autotuned context must
    hold the same particles as a context stepped as often with the default
    settings (a relaxation + projection case rides along in the same context
    and must stay finite and converged)."""
    mesh = W.unit_square(16, 0.2, periodic_x=True, seed_key=(0, 0, 0))
    params = W.default_params(mode=0, n_scalars=0, dt=1e-3, nu=1e-3)
    parts = W.init_particles(mesh, 30, 0, W.rng_for(0, 0, 7), u_std=0.1)
    F = W.frozen_fields(mesh, C0=2.1, omega=1.0, k=0.015)
    mesh2, params2, parts2 = _small_channel(ppe=10, ns=2, rtol=1e-12)
    _flush("[autotune] frozen-field case + relaxation case, one step per trial")
    sims = []
    for tune in (True, False):
        sim = P.Sim("fp64", "cuda:0")
        c1 = sim.add_case(mesh, params, len(parts["x"]))
        c2 = sim.add_case(mesh2, params2, len(parts2["x"]))
        sim.bind()
        sim.set_options(sort_interval=10, use_graph=True)
        sim.fields_upload(c1, F)
        sim.upload(c1, parts); sim.upload(c2, parts2)
        sim.init()
        sims.append((sim, c1, c2))
    r = sims[0][0].autotune(steps_per_trial=1)
    assert r["block_size"] in (64, 128, 256)
    assert r["sort_interval"] in (1, 2, 5, 10, 20)
    assert r["tail_rows"] in (0, 64, 256, 512, 1024, 2048)
    assert r["trials"] == 3 + 5 + 6 and r["ms_per_step"] > 0.0 and r["steps"] > 12
    sims[1][0].step(r["steps"])
    (a, a1, a2), (b, b1, b2) = sims
    n = len(parts["x"])
    A, B = _by_id(a.download(a1, n)), _by_id(b.download(b1, n))
    assert np.array_equal(A["elem"], B["elem"])
    for k in ("x", "y", "u", "v", "w", "omega"):
        assert np.array_equal(A[k], B[k]), k
    sa, sb = a.stats(a1), b.stats(b1)
    assert np.max(np.abs(sa - sb) / np.maximum(np.abs(sb), 1e-3)) <= 1e-10
    st2 = a.stats(a2)
    assert np.all(np.isfinite(st2))
    cnt = a.counters(a2)
    assert cnt["nan"] == 0 and cnt["cg_fail"] == 0


def test_row_parallel_phases_match_one_workgroup_completion(P):
    """The row-parallel phases (every level but the coarsest, tail_rows 0)
    apply the same preconditioner as the one-workgroup completion: the
    relaxation needs the same iterations either way, up to rounding, and
    reaches the same fields."""
    mesh = W.channel(n_half=24, nx=60, seed_key=(1, 2, 0))
    params = W.default_params(mode=2, dt=5e-4, nu=1.0 / 1080.0, n_scalars=0, dpdx=(-1.0, 0.0),
                              cg_rtol=1e-12, cg_maxit=20000, stream=1)
    parts = W.init_particles(mesh, 10, 0, W.rng_for(1, 2, 1), u_std=1.0)
    n = len(parts["x"])
    _flush(f"[phases_vs_completion] channel {mesh.n_elems} triangles, {n} particles")
    out = []
    for iters in (60, 1):
        sim = P.Sim("fp64", "cuda:0")
        cs = sim.add_case(mesh, params, n)
        sim.bind()
        sim.set_solver(iterations=iters, tail_rows=0)
        sim.upload(cs, parts)
        sim.init()
        sim.step(3)
        out.append((sim.counters(cs), sim.solver_info(), sim.fields(cs)))
    (ca, ia, Fa), (cb, ib, Fb) = out
    assert ia[1] >= 3, ia            # three levels ran as row-parallel phases
    assert ca["cg_fail"] == 0 and cb["cg_fail"] == 0
    assert abs(ca["cg_iters_er"] - cb["cg_iters_er"]) <= 5 * 4, (ca["cg_iters_er"], cb["cg_iters_er"])
    sc = np.maximum(np.abs(Fb).max(0), 1e-12)
    assert np.max(np.abs(Fa - Fb) / sc) <= 1e-8


def test_rebin_variant_follows_the_oracle(P, oracle_mod):
    """R-36 (bins and cell means formed again against the new fields at the
    end of each step), mode 1 on the small square with its scalar. The fields
    come from the statistics, whose summation order differs from the
    oracle's, so the comparison is to the bars of the other mode-1 runs:
    after one step the state to 1e-12 and the bins and cell counts equal
    (a bin flips only for |U - <U>| at rounding level), after 50 steps the
    statistics to 1e-9. In one context with a case that keeps the bins of its
    step, each case gives the same bits as alone (the rebinning pass skips
    the other case's tiles and elements)."""
    cfg = W.config_small()
    params = dict(cfg["params"], rebin=1)
    parts = cfg["particles"]
    n = len(parts["x"])
    _flush(f"[rebin] small square, {n} particles, bins formed again at the end of each step")
    sim, cs, o, oc = _pair(P, oracle_mod, cfg["mesh"], params, parts)
    sim.init(); o.init()
    sim.step(1); o.step(1)
    g, r = sim.download(cs, n), o.download(oc, n)
    assert np.array_equal(g["elem"], r["elem"])
    for k in ("x", "y", "u", "v", "w", "omega"):
        assert np.abs(g[k] - r[k]).max() <= 1e-12 * np.abs(r[k]).max(), k
    assert np.array_equal(g["bin"], r["bin"])
    gm, gc = sim.cell_means(cs)
    rm, rc = o.cell_means(oc)
    assert np.array_equal(gc, rc)
    np.testing.assert_allclose(gm, rm, rtol=1e-10, atol=1e-12)
    # the variant's bins are those of the new fields: they differ from the bins formed in the step
    sim.step(49); o.step(49)
    rows = _stat_rows(sim, cs)
    gst, rst = sim.stats(cs), o.stats(oc)
    d = np.abs(gst - rst)[rows] / _scale(rst, 1)[rows]
    assert d.max() <= 1e-9, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    # mixed with a case that keeps the bins of its step
    other = W.unit_square(10, 0.2, periodic_x=True, seed_key=(8, 0, 0))
    op = W.default_params(mode=1, n_scalars=2, dt=1e-3, nu=1e-3, stream=4, src=[(0.3, 0.3, 0.1, 1.0), (0.7, 0.6, 0.1, 1.0)])
    oparts = W.init_particles(other, 40, 2, W.rng_for(8, 0, 1), u_std=0.1)
    runs = []
    for group in ([(cfg["mesh"], params, parts), (other, op, oparts)], [(cfg["mesh"], params, parts)], [(other, op, oparts)]):
        s2 = P.Sim("fp64", "cuda:0")
        ids = [s2.add_case(m, p_, len(q["x"])) for m, p_, q in group]
        s2.bind()
        s2.set_options(sort_interval=3, use_graph=True)
        for i_, (m, p_, q) in zip(ids, group):
            s2.upload(i_, q)
        s2.init()
        s2.step(8)
        runs.append([(s2.download(i_, len(q["x"])), s2.cell_means(i_), s2.stats(i_)) for i_, (m, p_, q) in zip(ids, group)])
    for both, alone in ((runs[0][0], runs[1][0]), (runs[0][1], runs[2][0])):
        for k in both[0]:
            assert np.array_equal(both[0][k], alone[0][k]), k
        assert np.array_equal(both[1][0], alone[1][0]) and np.array_equal(both[1][1], alone[1][1])
        assert np.array_equal(both[2], alone[2])
