"""The boundary calls beside the plain step, through the C ABI: the device
draw of the initial ensemble (readings R-29..R-32) against the oracle's, the
stage mask of pdfmc_step against whole steps, and frozen field slots against
the oracle with the same slots frozen.

Bars: the initial draw is FP64 arithmetic on both sides in the same order
(Philox words, the project-written ln and sincos series, correctly rounded
sqrt), so the FP64 context matches the oracle bit for bit and the FP32
context holds the oracle's values rounded to float. A step taken in stages
equals the whole step bit for bit (the same kernels on the same inputs, with
the fixed summation order of the scatter). The frozen-slot run follows the
oracle to the 1e-9 bar of the 100-step parity runs.
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


def _init_cases():
    sq = W.unit_square(14, 0.2, periodic_x=True, periodic_y=False, seed_key=(2, 0, 0))
    ch = W.channel(n_half=8, nx=20, seed_key=(1, 2, 0))
    return [
        ("square-2scalars", sq, W.default_params(mode=1, n_scalars=2, stream=3), 37, 0.1, 0.25,
         [(0.5, 0.5, 0.2, 1.0), (0.25, 0.7, 0.15, 2.5)]),
        ("channel-1scalar", ch, W.default_params(mode=1, n_scalars=1, stream=0), 5, 1.0, 2.0,
         [(3.0, 1.0, 0.4, 1.0)]),
        ("square-no-scalars", sq, W.default_params(mode=0, n_scalars=0, stream=7), 1, 0.0, 1.0, []),
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(3), ids=[c[0] for c in _init_cases()])
def test_particles_init_matches_oracle(P, oracle_mod, precision, case):
    name, mesh, params, ppe, u_std, scale, disks = _init_cases()[case]
    n = mesh.n_elems * ppe
    _flush(f"[particles_init] {name} {precision}: {mesh.n_elems} triangles x {ppe} = {n} particles")
    sim = P.Sim(precision, "cuda:0")
    cs = sim.add_case(mesh, params, n + 17)
    sim.bind()
    assert sim.init_particles(cs, ppe, u_std=u_std, omega_scale=scale, disks=disks) == n
    g = sim.download(cs, n)
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, params)
    assert o.particles_init(oc, ppe, u_std=u_std, omega_scale=scale, disks=disks) == n
    r = o.download(oc, n)
    for k in ("elem", "id", "bin"):
        assert np.array_equal(g[k], r[k]), k
    for k in ("x", "y", "u", "v", "w", "omega", "weight", "psi"):
        want = r[k] if precision == "fp64" else r[k].astype(np.float32).astype(np.float64)
        assert np.array_equal(g[k], want), (k, np.max(np.abs(g[k] - want)))
    assert all(v == 0 for v in sim.counters(cs).values())
    # the drawn ensemble steps like an uploaded one
    sim.init()
    sim.step(3)
    assert sim.counters(cs)["nan"] == 0


def _stage_case():
    cfg = W.config_small()
    return cfg["mesh"], cfg["params"], cfg["particles"]


def _sim(P, mesh, params, parts, precision="fp64", use_graph=False):
    n = len(parts["x"])
    sim = P.Sim(precision, "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.set_options(sort_interval=0, use_graph=use_graph)
    sim.upload(cs, parts)
    sim.init()
    return sim, cs


def _state(sim, cs, n):
    mean, cnt = sim.cell_means(cs)
    return dict(parts=sim.download(cs, n), stats=sim.stats(cs), fields=sim.fields(cs), cmean=mean, ccnt=cnt)


def _same(a, b):
    if isinstance(a, dict):
        return all(_same(a[k], b[k]) for k in a)
    return np.array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stages_compose_to_the_whole_step(P, precision):
    """ADVANCE, then STATS, then FIELDS on one context equal one whole step on
    another, stage by stage; an empty mask changes nothing but the step
    index; after resetting the index both continue identically. The staged
    context replays captured graphs, the other launches eagerly."""
    mesh, params, parts = _stage_case()
    n = len(parts["x"])
    _flush(f"[stages] {precision} small square, {n} particles")
    a, ca = _sim(P, mesh, params, parts, precision, use_graph=True)
    b, cb = _sim(P, mesh, params, parts, precision)
    s0 = _state(a, ca, n)
    a.step(2, stages=0)
    assert _same(_state(a, ca, n), s0)
    a.set_step_index(0)
    b.step(1)
    s1 = _state(b, cb, n)
    assert not _same(s1["parts"], s0["parts"])
    a.step(1, stages=a.STAGE_ADVANCE)
    sa = _state(a, ca, n)
    assert _same(sa["parts"], s1["parts"])
    for k in ("stats", "fields", "cmean", "ccnt"):
        assert _same(sa[k], s0[k]), k
    a.step(1, stages=a.STAGE_STATS)
    sa = _state(a, ca, n)
    for k in ("parts", "stats", "cmean", "ccnt"):
        assert _same(sa[k], s1[k]), k
    assert _same(sa["fields"], s0["fields"])
    a.step(1, stages=a.STAGE_FIELDS)
    assert _same(_state(a, ca, n), s1)
    a.set_step_index(1)
    a.step(4)
    b.step(4)
    assert _same(_state(a, ca, n), _state(b, cb, n))
    assert a.counters(ca) == b.counters(cb)


def _stat_scale(rst):
    sc = np.abs(rst).copy()
    raw = rst[:, 5:8] + rst[:, 2:5] ** 2
    for c_, i in ((5, 0), (6, 1), (7, 2)):
        sc[:, c_] = raw[:, i]
    for c_, (i, j) in {8: (0, 1), 9: (0, 2), 10: (1, 2)}.items():
        sc[:, c_] = np.sqrt(raw[:, i] * raw[:, j])
    sc[:, 13] = rst[:, 13] + rst[:, 12] ** 2
    return np.maximum(sc, 1e-300)


def test_frozen_slots_follow_the_oracle(P, oracle_mod):
    """Mode 1 (fields from the statistics) with <omega>, C0 eps and the G_ij
    slots frozen at uploaded values, 40 steps, on both sides: the frozen
    slots keep the uploaded values bit for bit, the others are derived, and
    the run follows the oracle with the same freeze."""
    mesh, params, parts = _stage_case()
    n = len(parts["x"])
    F = W.frozen_fields(mesh, C0=3.5, omega=2.0, k=0.01, dpdx=(-1.0, 0.0))
    mask = sum(1 << q for q in range(14, 21))
    _flush(f"[freeze] small square, {n} particles, mask {mask:#x}, 40 steps")
    sim = P.Sim("fp64", "cuda:0")
    cs = sim.add_case(mesh, params, n)
    sim.bind()
    sim.fields_upload(cs, F, freeze_mask=mask)
    sim.upload(cs, parts)
    sim.init()
    sim.step(40)
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, params)
    o.fields_upload(oc, F, freeze_mask=mask)
    o.upload(oc, parts)
    o.init()
    o.step(40)
    gF, rF = sim.fields(cs), o.fields(oc)
    frozen = [q for q in range(22) if (mask >> q) & 1]
    assert np.array_equal(gF[:, frozen], F[:, frozen])
    assert np.array_equal(rF[:, frozen], F[:, frozen])
    assert not np.allclose(rF[:, 0], F[:, 0])          # <U_1> is derived
    _, sn = sim.case_info(cs)
    rows = np.unique(sn, return_index=True)[1]
    gst, rst = sim.stats(cs), o.stats(oc)
    d = (np.abs(gst - rst) / _stat_scale(rst))[rows]
    assert d.max() <= 1e-9, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    g, r = sim.download(cs, n), o.download(oc, n)
    assert (g["elem"] == r["elem"]).mean() > 0.999
    # a later upload without the mask lets every slot be derived again
    sim.fields_upload(cs, sim.fields(cs))
    sim.step(1)
    assert not np.array_equal(sim.fields(cs)[:, 19], F[:, 19])
