"""The particle advance and the full model between curved walls, through the
C ABI, against the FP64 oracle: an annulus whose two circles are polygons
with edges facing every direction (the general two-dimensional geometry of
Sec. I and Sec. III.B), the inner circle rotating, each of its edges a wall
of its own that moves along itself.

  - FP64, frozen random fields: after each of three steps the element ids,
    velocity bins and particle state equal the oracle's bit for bit and the
    walk counters are equal (R-12..R-14 reflect about each edge's own line
    and take that edge's wall velocity);
  - FP64, full model (Eqs. (4), (5), (9), the relaxation of R-19 with wall
    normals averaged over the edges at a node, the projection of R-27): the
    fields after the initial statistics and the statistics and fields after
    four steps, to the tolerances of the channel tests;
  - FP32, full model over 60 steps: every statistic within three standard
    errors of the oracle's at 99% of the (node, statistic) pairs.

The annulus has 800 triangles; 33 particles per element give 26,400
particles, 103 tiles of 256 with a ragged last tile.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _assert_state_equal, _pair, _scale, _stat_rows

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_1006_0549_amd as P
    return P


def _mesh():
    return W.annulus(n_r=8, n_theta=50, r0=0.5, r1=1.0, spin=1.0, seed_key=(6, 0, 0))


def test_annulus_frozen_bitwise(P, oracle_mod):
    mesh = _mesh()
    rng = np.random.default_rng(61)
    F = W.frozen_fields(mesh, C0=2.1, omega=1.3, k=0.02, dpdx=(0.3, -0.2))
    F[:, 0:3] = rng.normal(0, 0.05, (mesh.n_nodes, 3))
    F[:, 5:11] = rng.normal(0, 0.5, (mesh.n_nodes, 6))
    F[:, 11:14] = rng.normal(0, 1.0, (mesh.n_nodes, 3))
    F[:, 15:17] = rng.normal(0, 0.3, (mesh.n_nodes, 2))
    F[:, 21] = rng.normal(0.7, 0.1, mesh.n_nodes)
    params = W.default_params(mode=0, dt=2e-3, nu=2e-3, n_scalars=1, n_bins=8, dpdx=(0.3, -0.2),
                              src=[(0.0, 0.75, 0.1, 1.0)])
    parts = W.init_particles(mesh, 33, 1, rng, u_std=0.6, psi_disks=[(0.6, 0.0, 0.3, 1.0)])
    n = len(parts["x"])
    _flush(f"[annulus-frozen] {mesh.n_elems} triangles, {len(mesh.bcs)} walls, {n} particles, 3 steps, FP64")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, fields=F)
    sim.init(); o.init()
    for step in range(3):
        sim.step(1); o.step(1)
        g, r = sim.download(cs, n), o.download(oc, n)
        _assert_state_equal(g, r)
        assert np.array_equal(g["bin"], r["bin"])
        gst, rst = sim.stats(cs), o.stats(oc)
        rows = _stat_rows(sim, cs)
        d = np.abs(gst - rst)[rows] / _scale(rst, 1)[rows]
        assert d.max() <= 1e-12, (step, d.max())
    gc_, rc_ = sim.counters(cs), o.counters(oc)
    for k in ("walk_fallback", "reflect", "periodic", "omega_flip", "nan", "walk_steps"):
        assert gc_[k] == rc_[k], (k, gc_[k], rc_[k])
    assert rc_["reflect"] > 50 and rc_["walk_fallback"] == 0
    # reflections on both circles: particles within one step of either wall
    rad = np.hypot(g["x"], g["y"])
    assert (rad < 0.52).sum() > 0 and (rad > 0.98).sum() > 0


def _full(ns=1):
    mesh = _mesh()
    params = W.default_params(mode=2, dt=5e-4, nu=1e-3, n_scalars=ns, dpdx=(0.0, 0.0),
                              src=[(0.0, 0.75, 0.1, 1.0)][:ns], cg_rtol=1e-13, cg_maxit=20000, stream=3)
    parts = W.init_particles(mesh, 33, ns, W.rng_for(6, 0, 1), u_std=0.3)
    return mesh, params, parts


def test_annulus_full_model_fp64(P, oracle_mod):
    mesh, params, parts = _full()
    n = len(parts["x"])
    _flush(f"[annulus-full] {mesh.n_elems} triangles, {n} particles, mode 2, FP64")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts)
    sim.init(); o.init()
    rows = _stat_rows(sim, cs)
    gF, rF = sim.fields(cs)[rows], o.fields(oc)[rows]
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
    assert gc_["cg_fail"] == 0 and gc_["cg_iters_er"] > 0 and gc_["reflect"] > 0


def test_annulus_fp32_band(P, oracle_mod):
    from oracle import band
    mesh, params, parts = _full()
    n, steps = len(parts["x"]), 60
    _flush(f"[annulus-fp32-band] {n} particles, {steps} steps, FP32 against the FP64 oracle")
    sim, cs, o, oc = _pair(P, oracle_mod, mesh, params, parts, precision="fp32")
    sim.init(); o.init()
    sim.step(steps); o.step(steps)
    rows = _stat_rows(sim, cs)
    fr = band.fractions(sim.stats(cs), o.stats(oc), o.node_sums(oc), 1, rows=rows)
    _flush("[annulus-fp32-band] " + ", ".join(f"{k} {v['fraction']:.4f} (median {v['median_sigma']:.2g} sigma)"
                                             for k, v in fr.items()))
    for k, v in fr.items():
        assert v["fraction"] >= 0.99, (k, v)
        assert v["median_sigma"] < 0.5, (k, v)
