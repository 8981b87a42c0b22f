"""Pins of the oracle's particle equations (Eq.(2), (4), (5), (9)) and of the
grid statistics (Sec. I role (i), reading R-11).

With the Eulerian fields frozen (mode 0) each SDE reduces to a process whose
moments are known in closed form:
  - Eq.(4) with G constant, C0 eps = b^2, nu = 0: a vector Ornstein-Uhlenbeck
    process, E[U_{n+1}] = (I + dt G) E[U_n], Var recurrence of each component;
  - Eq.(4) with only the mean pressure gradient: U_n = U_0 - n dt grad<P>;
  - Eq.(2)+(4) viscous terms: E[dU_i] = 2 nu dt lap<U_i>, and, because the
    same dW_j drives both equations, Cov(dU_i, dX_j) = 2 nu dt d<U_i>/dx_j;
  - Eq.(5) with <omega>, S_omega frozen: mean recurrence
    m' = m (1 - C3 W dt - S W dt) + C3 W^2 dt; with S = 0 the stationary law
    is Gamma(1/C4, C4 W) (the CIR process), mean W, variance C4 W^2;
  - Eq.(9) with particles at rest: the cell sum of w psi is invariant and the
    cell variance is multiplied by (1 - dt/t_m)^2 each step.
The estimator is checked by partition of unity, conservation of the weighted
sums and a brute-force evaluation of the P1 shape functions by linear solves.
A run of the full model on a small channel guards the reading of the
projection (R-27), under which the channel stays bounded.
"""
import math

import numpy as np
import pytest

import workloads as W


def _box(n=16, periodic_y=True):
    return W.unit_square(n, 0.2, periodic_x=True, periodic_y=periodic_y)


def _frozen_run(oracle_mod, mesh, F, parts, steps, record=None, **kw):
    p = W.default_params(mode=0, nu=0.0, n_scalars=kw.pop("n_scalars", 0), n_bins=kw.pop("n_bins", 1), **kw)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, p)
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    out = []
    n = len(parts["x"])
    for s in range(steps):
        o.step(1)
        if record:
            out.append(o.download(cs, n))
    return o, cs, out


def _parts(mesh, ppe, seed, u0=(0.0, 0.0, 0.0), om0=1.0, ns=0):
    P = W.init_particles(mesh, ppe, ns, np.random.default_rng(seed))
    n = len(P["x"])
    P["u"][:], P["v"][:], P["w"][:] = u0
    P["omega"][:] = om0
    return P


def test_ou_mean_and_variance(oracle_mod):
    mesh = _box()
    a, b, dt = 2.0, 1.0, 0.05
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 14] = F[:, 17] = F[:, 18] = -a       # G11, G22, G33
    F[:, 15], F[:, 16] = 0.5, -0.3            # G12, G21 (not symmetric)
    F[:, 19] = 1.0
    F[:, 20] = b * b                          # C0 eps
    parts = _parts(mesh, 200, 11, u0=(1.0, -0.5, 1.0))
    N = len(parts["x"])
    steps = 12
    _, _, hist = _frozen_run(oracle_mod, mesh, F, parts, steps, record=True, dt=dt)
    G = np.array([[-a, 0.5], [-0.3, -a]])
    m = np.array([1.0, -0.5])
    m3, v3 = 1.0, 0.0
    vuv = np.zeros((2, 2))
    A = np.eye(2) + dt * G
    for s in range(steps):
        m = A @ m
        vuv = A @ vuv @ A.T + b * b * dt * np.eye(2)
        m3 = (1 - a * dt) * m3
        v3 = (1 - a * dt) ** 2 * v3 + b * b * dt
        U = np.stack([hist[s]["u"], hist[s]["v"]])
        se = np.sqrt(np.diag(vuv) / N)
        assert np.all(np.abs(U.mean(1) - m) < 4.5 * se), (s, U.mean(1), m)
        assert abs(hist[s]["w"].mean() - m3) < 4.5 * math.sqrt(v3 / N)
        # variance of w: standard error of a Gaussian sample variance
        assert abs(hist[s]["w"].var() - v3) < 4.5 * v3 * math.sqrt(2.0 / N)
        C = np.cov(U)
        assert np.all(np.abs(C - vuv) < 4.5 * np.sqrt(2.0 / N) * np.sqrt(np.outer(np.diag(vuv), np.diag(vuv))) + 1e-12)
    # lag-1 autocorrelation of w at the last step pair: 1 - a dt
    w1, w2 = hist[-2]["w"], hist[-1]["w"]
    r = np.corrcoef(w1, w2)[0, 1]
    # w2 = (1 - a dt) w1 + noise: r = (1 - a dt) sqrt(v1 / v2)
    r_exp = (1 - a * dt) * math.sqrt(w1.var() / w2.var())
    assert abs(r - r_exp) < 4.5 / math.sqrt(N)


def test_pressure_gradient_term_exact(oracle_mod):
    mesh = _box(10)
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 3], F[:, 4] = -1.0, 0.5
    parts = _parts(mesh, 5, 12, u0=(0.25, 0.0, -1.0))
    dt = 1e-3
    _, _, hist = _frozen_run(oracle_mod, mesh, F, parts, 7, record=True, dt=dt)
    u, v, w = hist[-1]["u"], hist[-1]["v"], hist[-1]["w"]
    assert np.allclose(u, 0.25 + 7 * dt, rtol=0, atol=1e-14)
    assert np.allclose(v, -0.5 * 7 * dt, rtol=0, atol=1e-14)
    assert np.all(w == -1.0)


def test_viscous_terms_share_the_wiener_increment(oracle_mod):
    mesh = _box()
    nu, dt = 1e-3, 0.05
    F = np.zeros((mesh.n_nodes, 22))
    dU = np.array([[0.3, 0.7], [-0.2, 0.1], [0.4, -0.5]])   # d<U_i>/dx_j
    F[:, 5:11] = dU.reshape(-1)
    F[:, 11:14] = (1.0, 2.0, 3.0)
    parts = _parts(mesh, 200, 13)
    N = len(parts["x"])
    x0, y0 = parts["x"].copy(), parts["y"].copy()
    p = W.default_params(mode=0, nu=nu, dt=dt, n_scalars=0, n_bins=1)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, p)
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    o.step(1)
    q = o.download(cs, N)
    dX = np.stack([q["x"] - x0, q["y"] - y0])
    dX -= np.round(dX)                      # periodic images
    dUs = np.stack([q["u"], q["v"], q["w"]])
    s2 = 2 * nu * dt
    for i in range(3):
        assert abs(dUs[i].mean() - s2 * F[0, 11 + i]) < 4.5 * math.sqrt(s2 * (dU[i] ** 2).sum() / N)
        for j in range(2):
            c = np.mean(dUs[i] * dX[j])
            var = s2 * s2 * ((dU[i] ** 2).sum() + dU[i, j] ** 2)
            assert abs(c - s2 * dU[i, j]) < 4.5 * math.sqrt(var / N), (i, j, c, s2 * dU[i, j])
    # the position increment itself is N(0, 2 nu dt)
    assert abs(dX.var(1) / s2 - 1).max() < 4.5 * math.sqrt(2.0 / N)


def test_frequency_mean_recurrence(oracle_mod):
    mesh = _box()
    Om, S, dt, C3, C4 = 2.0, 0.3, 0.005, 1.0, 0.25
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 19], F[:, 21] = Om, S
    parts = _parts(mesh, 200, 14, om0=1.0)
    N = len(parts["x"])
    _, cs_, hist = _frozen_run(oracle_mod, mesh, F, parts, 30, record=True, dt=dt, C3=C3, C4=C4)
    m = 1.0
    for s in range(30):
        m = m * (1 - C3 * Om * dt - S * Om * dt) + C3 * Om * Om * dt
        om = hist[s]["omega"]
        assert abs(om.mean() - m) < 4.5 * om.std() / math.sqrt(N) + 1e-12, (s, om.mean(), m)


def test_frequency_stationary_gamma(oracle_mod):
    mesh = _box(12)
    Om, dt, C3, C4 = 1.0, 0.01, 1.0, 0.25
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 19] = Om
    parts = _parts(mesh, 80, 15, om0=1.0)
    N = len(parts["x"])
    o, cs, _ = _frozen_run(oracle_mod, mesh, F, parts, 400, record=False, dt=dt, C3=C3, C4=C4)
    om = o.download(cs, N)["omega"]
    # Gamma(shape 1/C4, scale C4 Om): mean Om, variance C4 Om^2 (up to O(dt))
    assert abs(om.mean() - Om) < 4.5 * math.sqrt(C4 / N) + 0.01
    assert abs(om.var() / (C4 * Om * Om) - 1.0) < 4.5 * math.sqrt(2.0 / N) * 1.5 + 0.03
    from scipy import stats
    sk = stats.skew(om)
    assert abs(sk - 2 * math.sqrt(C4)) < 0.15


def test_iecm_conserves_cell_sums_and_decays_variance(oracle_mod):
    mesh = _box(10)
    dt, Cphi = 0.05, 2.0
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 19] = 1.5                     # <omega>: 1/t_m = Cphi/2 * 1.5
    rng = np.random.default_rng(16)
    parts = _parts(mesh, 60, 16, ns=2)
    N = len(parts["x"])
    # tiny frozen velocities: particles stay put, bins are the octants of U
    parts["u"], parts["v"], parts["w"] = (rng.standard_normal((3, N)) * 1e-13)
    parts["psi"] = rng.random((2, N))
    for nb in (8, 1):
        o = oracle_mod.Oracle()
        cs = o.add_case(mesh, W.default_params(mode=0, nu=0.0, dt=dt, Cphi=Cphi, n_scalars=2, n_bins=nb))
        o.fields_upload(cs, F)
        o.upload(cs, parts)
        o.init()
        q0 = o.download(cs, N)
        _, cnt = o.cell_means(cs)
        o.step(1)
        q1 = o.download(cs, N)
        assert np.array_equal(q0["elem"], q1["elem"])
        f = dt * 0.5 * Cphi * 1.5
        e, b = q0["elem"], q0["bin"].astype(np.int64)
        # cells: (e, b) when that bin holds >= n_min particles, else the residual of e
        big = cnt[e, b] >= 4
        cell = np.where(big, e * 9 + b, e * 9 + 8)
        for a in range(2):
            w = q0["weight"]
            s0 = np.bincount(cell, w * q0["psi"][a])
            s1 = np.bincount(cell, w * q1["psi"][a])
            assert np.allclose(s0, s1, rtol=1e-13, atol=1e-16)
            sw = np.bincount(cell, w)
            m = np.divide(s0, sw, out=np.zeros_like(s0), where=sw > 0)
            v0 = np.bincount(cell, w * (q0["psi"][a] - m[cell]) ** 2)
            v1 = np.bincount(cell, w * (q1["psi"][a] - m[cell]) ** 2)
            assert np.allclose(v1, (1 - f) ** 2 * v0, rtol=1e-11, atol=1e-15)
        if nb == 1:
            assert np.all(q0["bin"] == 0)
        else:
            octant = (parts["u"] >= 0) * 1 + (parts["v"] >= 0) * 2 + (parts["w"] >= 0) * 4
            assert np.array_equal(q0["bin"], octant)


def test_sources_set_value_inside_disk(oracle_mod):
    mesh = _box(12, periodic_y=False)
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 19] = 1.0
    parts = _parts(mesh, 30, 17, ns=2)
    N = len(parts["x"])
    src = [(0.4, 0.5, 0.15, 1.0), (0.7, 0.3, 0.1, 2.5)]
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, nu=1e-3, dt=1e-3, n_scalars=2, src=src))
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    o.step(1)
    q = o.download(cs, N)
    for a, (cx, cy, r, val) in enumerate(src):
        inside = (q["x"] - cx) ** 2 + (q["y"] - cy) ** 2 < r * r
        assert inside.sum() > 10
        assert np.all(q["psi"][a][inside] == val)
        assert np.all(q["psi"][a][~inside] == 0.0)


# ---------------------------------------------------------------- estimator

def _stat_rows(o, cs):
    info = o.mesh_info(cs)
    return np.unique(info["stat_node"], return_index=True)[1]


def test_estimator_partition_and_conservation(oracle_mod):
    cfg = W.config_small()
    o = oracle_mod.Oracle()
    cs = o.add_case(cfg["mesh"], cfg["params"])
    o.upload(cs, cfg["particles"])
    o.init()
    o.step(3)
    q = o.download(cs, len(cfg["particles"]["x"]))
    rows = _stat_rows(o, cs)
    S = o.node_sums(cs)[rows]
    w = q["weight"]
    assert abs(S[:, 0].sum() - w.sum()) < 1e-13 * w.sum()
    for col, Q in [(1, q["u"]), (2, q["v"]), (3, q["w"]), (4, q["u"] ** 2), (7, q["u"] * q["v"]),
                   (10, q["omega"]), (11, q["psi"][0]), (12, q["psi"][0] ** 2)]:
        ref = (w * Q).sum()
        assert abs(S[:, col].sum() - ref) <= 1e-12 * max(1e-30, (w * np.abs(Q)).sum()), col
    st = o.stats(cs)[rows]
    info = o.mesh_info(cs)
    assert np.allclose(st[:, 1], st[:, 0] / info["vol"][rows], rtol=1e-14)
    # density of a uniform ensemble is 1 on average (non-hybrid consistency)
    assert abs(np.average(st[:, 1], weights=info["vol"][rows]) - 1.0) < 1e-12


def test_estimator_brute_force_shape_functions(oracle_mod):
    mesh = W.unit_square(5, 0.2, periodic_x=True)
    parts = W.init_particles(mesh, 7, 1, np.random.default_rng(18), u_std=1.0,
                             psi_disks=[(0.5, 0.5, 0.3, 1.0)])
    F = np.zeros((mesh.n_nodes, 22))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=1))
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    info = o.mesh_info(cs)
    sn = info["stat_node"]
    nsn = info["n_stat_nodes"]
    N = len(parts["x"])
    # shape functions by solving [x_k; y_k; 1] lam = [x; y; 1]
    Wn = np.zeros(nsn)
    Qs = np.stack([parts["u"], parts["v"], parts["w"], parts["omega"], parts["psi"][0]])
    SQ = np.zeros((5, nsn))
    for p in range(N):
        e = parts["elem"][p]
        P = mesh.xy[mesh.tri[e]]
        A = np.vstack([P.T, np.ones(3)])
        lam = np.linalg.solve(A, [parts["x"][p], parts["y"][p], 1.0])
        for k in range(3):
            s = sn[mesh.tri[e, k]]
            Wn[s] += parts["weight"][p] * lam[k]
            SQ[:, s] += parts["weight"][p] * lam[k] * Qs[:, p]
    means = SQ / Wn
    cov = np.zeros(nsn)
    for p in range(N):
        e = parts["elem"][p]
        P = mesh.xy[mesh.tri[e]]
        lam = np.linalg.solve(np.vstack([P.T, np.ones(3)]), [parts["x"][p], parts["y"][p], 1.0])
        for k in range(3):
            s = sn[mesh.tri[e, k]]
            cov[s] += parts["weight"][p] * lam[k] * (parts["u"][p] - means[0, s]) * (parts["v"][p] - means[1, s])
    cov /= Wn
    st = o.stats(cs)
    rows = np.unique(sn, return_index=True)[1]
    st = st[rows]
    assert np.allclose(st[:, 0], Wn, rtol=1e-12)
    for j, col in enumerate([2, 3, 4, 11, 12]):
        assert np.allclose(st[:, col], means[j], rtol=1e-11, atol=1e-14)
    assert np.allclose(st[:, 8], cov, rtol=1e-10, atol=1e-14)


def test_estimator_constant_field(oracle_mod):
    mesh = _box(8, periodic_y=False)
    parts = _parts(mesh, 20, 19, u0=(1.5, -2.0, 0.25), om0=3.0)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=0))
    o.fields_upload(cs, np.zeros((mesh.n_nodes, 22)))
    o.upload(cs, parts)
    o.init()
    st = o.stats(cs)
    assert np.allclose(st[:, 2:5], [1.5, -2.0, 0.25], rtol=1e-14)
    assert np.allclose(st[:, 11], 3.0, rtol=1e-14)
    assert np.abs(st[:, 5:11]).max() < 1e-28


def test_thin_nodes_keep_previous_moments(oracle_mod):
    """R-34: the effective sample size W^2 / sum (w N)^2 of each node, from
    brute-force shape functions, against the oracle's node sums. The first
    statistics take every node's estimate; afterwards nodes below n_eff_min
    keep their previous moments while W and the density are updated."""
    mesh = W.unit_square(6, 0.2, periodic_x=False)
    rng = np.random.default_rng(23)
    parts = W.init_particles(mesh, 5, 0, rng, u_std=1.0)
    parts["weight"] = parts["weight"] * rng.uniform(0.2, 5.0, size=len(parts["x"]))   # uneven weights
    Wn = np.zeros(mesh.n_nodes)
    W2 = np.zeros(mesh.n_nodes)
    for p in range(len(parts["x"])):
        e = parts["elem"][p]
        P = mesh.xy[mesh.tri[e]]
        lam = np.linalg.solve(np.vstack([P.T, np.ones(3)]), [parts["x"][p], parts["y"][p], 1.0])
        for k in range(3):
            wn = parts["weight"][p] * lam[k]
            Wn[mesh.tri[e, k]] += wn
            W2[mesh.tri[e, k]] += wn * wn
    neff = Wn ** 2 / W2
    thr = float(np.median(neff))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=0, n_eff_min=thr))
    o.fields_upload(cs, np.zeros((mesh.n_nodes, 22)))
    o.upload(cs, parts)
    o.init()
    S = o.node_sums(cs)
    assert np.allclose(S[:, -1], W2, rtol=1e-12)
    st1 = o.stats(cs)
    assert o.counters(cs)["empty_node"] == 0          # first statistics: every node estimated
    # same positions and weights, new velocities: thin nodes keep st1's moments
    parts2 = dict(parts)
    for key in ("u", "v", "w"):
        parts2[key] = rng.normal(0.0, 1.0, size=len(parts["x"]))
    o.upload(cs, parts2)
    o.init()
    st2 = o.stats(cs)
    thin = neff < thr
    assert 0 < thin.sum() < mesh.n_nodes
    assert np.allclose(st2[:, 0], Wn, rtol=1e-12)
    assert np.array_equal(st2[thin, 2:], st1[thin, 2:])
    assert np.all(np.abs(st2[~thin, 2:5] - st1[~thin, 2:5]).sum(1) > 0.0)
    assert o.counters(cs)["empty_node"] == int(thin.sum())


def _reaction_case(oracle_mod, mesh, parts, ns, reaction, k, dt, steps, n_bins=8):
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 19] = 1.5
    p = W.default_params(mode=0, nu=0.0, dt=dt, n_scalars=ns, n_bins=n_bins, reaction=reaction, k_react=k)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, p)
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    N = len(parts["x"])
    out = [o.download(cs, N)]
    for _ in range(steps):
        o.step(1)
        out.append(o.download(cs, N))
    return out


def _resting(mesh, ppe, seed, ns):
    parts = _parts(mesh, ppe, seed, ns=ns)
    rng = np.random.default_rng(seed + 1)
    N = len(parts["x"])
    parts["u"], parts["v"], parts["w"] = rng.standard_normal((3, N)) * 1e-13
    return parts, rng, N


def test_reaction_first_order_decay_closed_form(oracle_mod):
    """Eq.(9) with S_a = -k_a psi_a (R-35). A uniform composition does not
    mix, so every particle follows the forward-Euler recursion
    psi_n = psi_0 (1 - k dt)^n, which lies below exp(-k t) by at most
    n (k dt)^2 / 2. With a random composition the IECM step conserves the
    mass-weighted sum, so that sum decays by exactly (1 - k dt) per step."""
    mesh = _box(10)
    dt, k, steps = 0.01, (2.0, 0.5), 40
    parts, rng, N = _resting(mesh, 30, 31, 2)
    parts["psi"] = np.stack([np.full(N, 1.0), np.full(N, 0.6)])
    out = _reaction_case(oracle_mod, mesh, parts, 2, 1, k + (0.0, 0.0), dt, steps)
    for a in range(2):
        h = k[a] * dt
        want = parts["psi"][a][0] * (1.0 - h) ** steps
        assert np.allclose(out[-1]["psi"][a], want, rtol=1e-12, atol=0)
        exact = parts["psi"][a][0] * math.exp(-k[a] * dt * steps)
        gap = exact - out[-1]["psi"][a]
        assert np.all(gap >= 0) and np.all(gap <= parts["psi"][a][0] * steps * h * h / 2)
    parts["psi"] = rng.random((2, N))
    out = _reaction_case(oracle_mod, mesh, parts, 2, 1, k + (0.0, 0.0), dt, 10)
    w = parts["weight"]
    for a in range(2):
        s = np.array([np.sum(w * q["psi"][a]) for q in out])
        assert np.allclose(s[1:] / s[:-1], 1.0 - k[a] * dt, rtol=1e-12, atol=0)
        # the scalar still mixes: its weighted variance falls faster than the mean squared
        m = s / np.sum(w)
        var = np.array([np.sum(w * (q["psi"][a] - mm) ** 2) for q, mm in zip(out, m)])
        assert var[-1] / var[0] < (1.0 - k[a] * dt) ** 20


def test_reaction_a_plus_b_invariants(oracle_mod):
    """A + B -> P at the rate k psi_A psi_B (R-35). Mixing conserves every
    mass-weighted sum, the reaction consumes A and B at the same rate and
    produces P at that rate: sum w (A + P) and sum w (B + P) are invariant,
    and sum w A falls by exactly dt k sum w A B over a step. A uniform
    composition follows a_{n+1} = a_n - dt k a_n^2, within O(dt) of the exact
    a_0 / (1 + k a_0 t)."""
    mesh = _box(10)
    dt, k = 0.01, 3.0
    parts, rng, N = _resting(mesh, 30, 37, 3)
    parts["psi"] = np.stack([0.5 + 0.5 * rng.random(N), 0.2 + 0.6 * rng.random(N), np.zeros(N)])
    out = _reaction_case(oracle_mod, mesh, parts, 3, 2, (k, 0.0, 0.0, 0.0), dt, 3)
    w = parts["weight"]
    for q0, q1 in zip(out[:-1], out[1:]):
        A0, B0, P0 = q0["psi"]
        A1, B1, P1 = q1["psi"]
        assert np.isclose(np.sum(w * (A1 + P1)), np.sum(w * (A0 + P0)), rtol=1e-13, atol=0)
        assert np.isclose(np.sum(w * (B1 + P1)), np.sum(w * (B0 + P0)), rtol=1e-13, atol=0)
        drop = np.sum(w * A0) - np.sum(w * A1)
        assert np.isclose(drop, dt * k * np.sum(w * A0 * B0), rtol=1e-9, atol=0)
        assert np.all(P1 >= P0)
    steps, a0 = 30, 0.8
    parts["psi"] = np.stack([np.full(N, a0), np.full(N, a0), np.zeros(N)])
    out = _reaction_case(oracle_mod, mesh, parts, 3, 2, (k, 0.0, 0.0, 0.0), dt, steps)
    a = a0
    for n in range(1, steps + 1):
        a = a - dt * k * a * a
        assert np.allclose(out[n]["psi"][0], a, rtol=1e-12, atol=0)
        assert np.allclose(out[n]["psi"][1], a, rtol=1e-12, atol=0)
        assert np.allclose(out[n]["psi"][2], a0 - a, rtol=1e-11, atol=1e-15)
    t = steps * dt
    assert abs(a - a0 / (1 + k * a0 * t)) < 2 * dt * (k * a0) ** 2 * t


def test_reaction_rejections(oracle_mod):
    mesh = _box(6)
    o = oracle_mod.Oracle()
    for bad in (dict(reaction=3), dict(reaction=2, n_scalars=2), dict(reaction=1, k_react=(-1.0, 0, 0, 0))):
        p = W.default_params(mode=0, **{"n_scalars": 3, **bad})
        with pytest.raises(RuntimeError):
            o.add_case(mesh, p)
    # reaction 0 ignores the rate constants
    parts, rng, N = _resting(mesh, 20, 41, 1)
    parts["psi"] = rng.random((1, N))
    a = _reaction_case(oracle_mod, mesh, parts, 1, 0, (5.0, 0, 0, 0), 0.01, 3)
    b = _reaction_case(oracle_mod, mesh, parts, 1, 0, (0.0, 0, 0, 0), 0.01, 3)
    assert np.array_equal(a[-1]["psi"], b[-1]["psi"])


def test_full_model_channel_stays_bounded(oracle_mod):
    """Regression for the reading of the projection (R-27, Sec. II closing
    paragraph): the full model (elliptic relaxation and projection) on a small
    channel, 20 particles per element, 250 steps. With the non-incremental
    projection (<P> = phi, particles corrected by -dt grad <P> at the next
    step) velocities and stresses stay at their initial scale. The incremental
    form (<P> += phi through the next predictor) fed the sampling noise of <U>
    into <P> with no damping: on this channel it reached max|U| ~ 50 and node
    <v'^2> ~ 400 by step 180, and its relaxation solve stopped converging at
    step 289."""
    mesh = W.channel(n_half=10, nx=24, seed_key=(1, 1, 0))
    params = W.default_params(mode=2, dt=5e-4, nu=1.0 / 1080.0, n_scalars=0, dpdx=(-1.0, 0.0), stream=1)
    parts = W.init_particles(mesh, 20, 0, W.rng_for(1, 1, 1), u_std=1.0)
    n = len(parts["x"])
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.init()
    for _ in range(5):
        o.step(50)
        r = o.download(cs, n)
        st = o.stats(cs)
        umax = float(np.abs(np.stack([r["u"], r["v"], r["w"]])).max())
        assert np.all(np.isfinite(st)) and umax < 8.0, umax
        assert st[:, 5:8].max() < 6.0, st[:, 5:8].max()
        assert np.abs(o.pressure(cs)).max() < 100.0
    cnt = o.counters(cs)
    assert cnt["nan"] == 0 and cnt["cg_fail"] == 0
