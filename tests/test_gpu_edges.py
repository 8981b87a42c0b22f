"""Degenerate inputs of the particle path against the FP64 oracle, through the
C ABI:

  - thin statistics nodes (R-34): the first statistics take every node's
    estimate; after a second ensemble is uploaded on the same positions,
    nodes whose effective sample size W^2 / sum (w N)^2 falls below n_eff_min
    keep their previous moments, bit for bit, while W and the density follow
    the new sums, and the empty-node counter equals the oracle's;
  - a batch holding a case of one particle (one tile with 255 idle lanes)
    and a case with no particles at all beside an ordinary case: three
    frozen-field steps give the oracle's state bit for bit in every case, the
    same counters, and for the empty case all-zero statistics (every node
    empty keeps the zero moments it started with).
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _assert_state_equal, _scale, _stat_rows

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_1006_0549_amd as P
    return P


def _brute_neff(mesh, parts):
    Wn = np.zeros(mesh.n_nodes)
    W2 = np.zeros(mesh.n_nodes)
    for p in range(len(parts["x"])):
        e = parts["elem"][p]
        Pv = mesh.xy[mesh.tri[e]]
        lam = np.linalg.solve(np.vstack([Pv.T, np.ones(3)]), [parts["x"][p], parts["y"][p], 1.0])
        for k in range(3):
            wn = parts["weight"][p] * lam[k]
            Wn[mesh.tri[e, k]] += wn
            W2[mesh.tri[e, k]] += wn * wn
    return Wn ** 2 / W2


def test_thin_nodes_follow_the_oracle(P, oracle_mod):
    mesh = W.unit_square(9, 0.2, periodic_x=False, seed_key=(71, 0, 0))
    rng = np.random.default_rng(71)
    parts = W.init_particles(mesh, 5, 0, rng, u_std=1.0)
    parts["weight"] = parts["weight"] * rng.uniform(0.2, 5.0, size=len(parts["x"]))
    neff = np.sort(_brute_neff(mesh, parts))
    k = len(neff) // 2
    assert neff[k + 1] - neff[k] > 1e-6 * neff[k]
    thr = 0.5 * (neff[k] + neff[k + 1])          # no node within rounding of the threshold
    params = W.default_params(mode=0, n_scalars=0, n_eff_min=float(thr))
    F = np.zeros((mesh.n_nodes, 22))
    n = len(parts["x"])
    _flush(f"[thin-nodes] {mesh.n_nodes} nodes, {n} particles, n_eff_min {thr:.3f}, FP64")
    sim = P.Sim("fp64", "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.fields_upload(cs, F)
    sim.upload(cs, parts)
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, params)
    o.fields_upload(oc, F)
    o.upload(oc, parts)
    sim.init(); o.init()
    rows = _stat_rows(sim, cs)
    g1, r1 = sim.stats(cs), o.stats(oc)
    d = np.abs(g1 - r1)[rows] / _scale(r1, 0)[rows]
    assert d.max() <= 1e-12, d.max()
    assert sim.counters(cs)["empty_node"] == o.counters(oc)["empty_node"] == 0
    parts2 = dict(parts)
    for key in ("u", "v", "w"):
        parts2[key] = rng.normal(0.0, 1.0, size=n)
    sim.upload(cs, parts2); o.upload(oc, parts2)
    sim.init(); o.init()
    g2, r2 = sim.stats(cs), o.stats(oc)
    thin_o = np.all(r2[:, 2:] == r1[:, 2:], axis=1)[rows]
    thin_g = np.all(g2[:, 2:] == g1[:, 2:], axis=1)[rows]
    assert 0 < thin_o.sum() < len(rows)
    assert np.array_equal(thin_g, thin_o)
    d = np.abs(g2 - r2)[rows] / _scale(r2, 0)[rows]
    assert d.max() <= 1e-12, d.max()
    assert sim.counters(cs)["empty_node"] == o.counters(oc)["empty_node"] == int(thin_o.sum())


def _subset(parts, m):
    return {k: (v[:m].copy() if v.ndim == 1 else v[:, :m].copy()) for k, v in parts.items()}


def test_one_particle_and_empty_cases_in_a_batch(P, oracle_mod):
    from test_gpu_parity import _frozen_case
    mesh, params, parts, F = _frozen_case(ns=1, nb=8)
    one = _subset(W.init_particles(mesh, 1, 1, np.random.default_rng(72), u_std=0.4,
                                   psi_disks=[(0.5, 0.5, 0.25, 1.0)]), 1)
    none = _subset(parts, 0)
    ensembles = [parts, one, none]
    _flush(f"[edge-batch] cases of {[len(e['x']) for e in ensembles]} particles, 3 frozen steps, FP64")
    sim = P.Sim("fp64", "cuda:0")
    o = oracle_mod.Oracle()
    cases = [(sim.add_case(mesh, params, len(e["x"])), o.add_case(mesh, params)) for e in ensembles]
    sim.bind()
    for (cs, oc), e in zip(cases, ensembles):
        sim.fields_upload(cs, F); o.fields_upload(oc, F)
        sim.upload(cs, e); o.upload(oc, e)
    sim.init(); o.init()
    for step in range(3):
        sim.step(1); o.step(1)
        for (cs, oc), e in zip(cases, ensembles):
            n = len(e["x"])
            if n:
                g, r = sim.download(cs, n), o.download(oc, n)
                _assert_state_equal(g, r)
                assert np.array_equal(g["bin"], r["bin"])
            rows = _stat_rows(sim, cs)
            gst, rst = sim.stats(cs), o.stats(oc)
            assert np.isfinite(gst).all()
            d = np.abs(gst - rst)[rows] / _scale(rst, 1)[rows]
            assert d.max() <= 1e-12, (step, n, d.max())
    for (cs, oc), e in zip(cases, ensembles):
        gc_, rc_ = sim.counters(cs), o.counters(oc)
        for k in ("walk_fallback", "reflect", "periodic", "omega_flip", "nan", "walk_steps", "empty_node"):
            assert gc_[k] == rc_[k], (len(e["x"]), k, gc_[k], rc_[k])
    empty = sim.stats(cases[2][0])
    assert not empty.any()
