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
    empty keeps the zero moments it started with);
  - elements with records in more workgroups than their 64 list entries
    (particles spread one per workgroup): the further records go through the
    pass's overflow list and are summed in key order like the others, so
    nothing falls back to atomics, two runs agree bit for bit, and the FP64
    sums match the oracle's.
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


def _spread_case(seed=73):
    """The small square (450 elements) with 100 particles of each of
    elements 0, 1 and 2 spread one per workgroup: workgroup w starts with the
    w-th particle of each of the three, then 253 of the other elements'
    particles in element order. Each of the three elements then has a record
    in each of 100 workgroups, more than its 64 list entries."""
    mesh = W.unit_square(16, 0.2, periodic_x=True, periodic_y=False, seed_key=(73, 0, 0))
    rng = np.random.default_rng(seed)
    base = W.init_particles(mesh, 60, 1, rng, u_std=0.3, psi_disks=[(0.5, 0.5, 0.25, 1.0)])
    dense = W.init_particles(mesh, 100, 1, rng, u_std=0.3, psi_disks=[(0.5, 0.5, 0.25, 1.0)])
    heads = [np.nonzero(dense["elem"] == el)[0] for el in range(3)]
    rest = np.nonzero(base["elem"] >= 3)[0]
    order = []
    for w in range(100):
        order += [("d", heads[el][w]) for el in range(3)]
        order += [("b", r) for r in rest[253 * w:253 * (w + 1)]]
    order += [("b", r) for r in rest[253 * 100:]]
    parts = {}
    for key in base:
        col = [dense[key][..., i] if src == "d" else base[key][..., i] for src, i in order]
        parts[key] = np.stack(col, axis=-1) if base[key].ndim == 2 else np.array(col, dtype=base[key].dtype)
    parts["id"] = np.arange(len(order), dtype=np.uint32)
    F = W.frozen_fields(mesh, C0=2.1, omega=1.3, k=0.02)
    params = W.default_params(mode=0, dt=2e-3, nu=2e-3, n_scalars=1, n_bins=8, src=[])
    return mesh, params, parts, F


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_elements_with_more_records_than_their_list(P, oracle_mod, precision):
    """Elements whose particles lie in more workgroups than the 64 list
    entries of an element: their further records go through the pass's
    overflow list and are still summed in key order, so no sum falls back to
    atomics (scatter_overflow stays 0), two runs give the same bits, and the
    FP64 node sums and statistics match the oracle to the bar of a listed
    element."""
    mesh, params, parts, F = _spread_case()
    n = len(parts["x"])
    _flush(f"[spread] {precision}: {n} particles, elements 0-2 spread one particle per workgroup, 2 frozen steps")

    def run():
        sim = P.Sim(precision, "cuda:0")
        cs = sim.add_case(mesh, params, n)
        sim.bind()
        sim.fields_upload(cs, F)
        sim.upload(cs, parts)
        sim.init()
        sim.step(2)
        return sim, cs

    s1, c1 = run()
    s2, c2 = run()
    assert s1.counters(c1)["scatter_overflow"] == 0
    assert np.array_equal(s1.node_sums(c1), s2.node_sums(c2))
    assert np.array_equal(s1.stats(c1), s2.stats(c2))
    if precision == "fp64":
        o = oracle_mod.Oracle()
        oc = o.add_case(mesh, params)
        o.fields_upload(oc, F)
        o.upload(oc, parts)
        o.init(); o.step(2)
        _assert_state_equal(s1.download(c1, n), o.download(oc, n))
        gs, rs = s1.node_sums(c1), o.node_sums(oc)
        tol = 1e-13 * np.abs(rs).max(0) + 1e-300
        assert np.all(np.abs(gs - rs) <= np.maximum(tol, 1e-13 * np.abs(rs))), np.max(np.abs(gs - rs))
        rows = _stat_rows(s1, c1)
        d = np.abs(s1.stats(c1) - o.stats(oc))[rows] / _scale(o.stats(oc), 1)[rows]
        assert d.max() <= 1e-12, d.max()
