"""Closed-form pins of the oracle parts that the earlier pins left open.

Each test ties an oracle function to something other than the oracle itself
(a special case with a hand-derived answer, a limit, a textbook definition or
brute force), chosen so that a plausible mistake (a sign, a transposed index,
a vertex paired with the wrong shape function, a missing clamp) fails it:

  - P1 interpolation (R-06) through a frozen linear mean velocity: with
    G_ij = -g delta_ij and no other forcing, Eq.(4) gives
    U^{n+1} = U - g dt (U - <U>(X^n)) with <U> linear in x, y exactly;
  - production and S_omega of Eq.(6) under homogeneous shear;
  - the elliptic-relaxation source of R-19 under simple shear, its A_v and
    length-scale limits, and its isotropic part, wall values, G_ij and C0 eps
    through the whole derivation on a periodic box and on a walled square;
  - the mixing clamp dt/t_m <= 1 of R-24;
  - the decay of k under the simplified Langevin model (R-20);
  - the walk cap (R-12) and the reflection cap (R-14) falling back to the
    brute-force search of R-13.
"""
import math

import numpy as np
import pytest

import workloads as W

# statistics columns (orc_stats layout)
W_, RHO, U1, U2, U3, R11, R22, R33, R12, R13, R23, OM = range(12)
# field slots (R-06 list)
F_U1, F_DPX, F_DPY, F_G11, F_G12, F_G21, F_G22, F_G33, F_OMEGA, F_C0EPS, F_SOMEGA = 0, 3, 4, 14, 15, 16, 17, 18, 19, 20, 21


def _stats(mesh, ns, U, R, om):
    """Node statistics: U (n_nodes, 3), R = (r11, r22, r33, r12, r13, r23), om."""
    st = np.zeros((mesh.n_nodes, 12 + 2 * ns))
    st[:, W_] = 1.0
    st[:, RHO] = 1.0
    st[:, U1:U3 + 1] = U
    st[:, R11:R23 + 1] = R
    st[:, OM] = om
    return st


def _derive(oracle_mod, mesh, params, stats, project=False):
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.set_stats(cs, stats)
    o.derive(cs, project)
    return o.fields(cs)


# ------------------------------------------------------------ interpolation

def test_interpolation_reproduces_a_linear_mean_velocity(oracle_mod):
    """Frozen fields <U_i> = a_i + b_i x + c_i y, G_ij = -g delta_ij, no
    pressure gradient, viscosity or C0 eps: Eq.(4) by forward Euler gives
    U^{n+1} = U - g dt (U - <U>(X^n)) for every particle (R-03, R-06)."""
    mesh = W.unit_square(9, 0.2, periodic_x=False, periodic_y=False, seed_key=(90, 0, 0))
    g, dt = 3.0, 1e-3
    a = np.array([0.3, -0.2, 0.5])
    b = np.array([1.1, -0.7, 0.4])
    c = np.array([-0.6, 0.9, 1.3])
    F = np.zeros((mesh.n_nodes, 22))
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    for i in range(3):
        F[:, F_U1 + i] = a[i] + b[i] * x + c[i] * y
    F[:, F_G11] = F[:, F_G22] = F[:, F_G33] = -g
    F[:, F_OMEGA] = 1.0
    params = W.default_params(mode=0, dt=dt, nu=0.0, n_scalars=0, dpdx=(0.0, 0.0))
    parts = W.init_particles(mesh, 20, 0, W.rng_for(90, 0, 1), u_std=0.3)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.fields_upload(cs, F)
    o.init()
    o.step(1)
    r = o.download(cs, len(parts["x"]))
    x0, y0 = parts["x"], parts["y"]
    # particles that cannot have reached a wall in one step keep their velocity sign
    inside = np.minimum.reduce([x0, 1 - x0, y0, 1 - y0]) > 5e-3
    assert inside.sum() > 0.8 * len(x0)
    for i, k in enumerate(("u", "v", "w")):
        mean = a[i] + b[i] * x0 + c[i] * y0
        want = parts[k] - g * dt * (parts[k] - mean)
        np.testing.assert_allclose(r[k][inside], want[inside], rtol=0, atol=1e-14)
    # and the positions moved by U^n dt exactly (Eq.(2) with nu = 0)
    np.testing.assert_allclose(r["x"][inside], (x0 + parts["u"] * dt)[inside], rtol=0, atol=1e-15)


# ------------------------------------------------------------ Eq.(6)

@pytest.mark.parametrize("periodic", [True, False])
def test_production_and_somega_under_homogeneous_shear(oracle_mod, periodic):
    """<U_1> = S y and <U_3> = S3 y (plus, on the walled square, <U_2> = T x
    and <U_3> += S4 x): production P = -<u_i u_j> d<U_i>/dx_j reduces to
    -(u12 S + u23 S3 [+ u12 T + u13 S4]); S_omega = Cw2 - Cw1 P / eps with
    eps = k <omega> (Eq.(6)). The recovered gradients are exact for linear
    fields (R-16), so the closed form holds at every node."""
    mesh = W.unit_square(9, 0.2, periodic_x=periodic, periodic_y=False, seed_key=(91, 0, 0))
    S, S3, T, S4 = 2.5, -1.5, 0.8, 1.7
    r11, r22, r33, r12, r13, r23 = 0.9, 0.4, 0.6, -0.23, 0.11, 0.17
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    U = np.zeros((mesh.n_nodes, 3))
    U[:, 0] = S * y
    U[:, 2] = S3 * y
    prod = -(r12 * S + r23 * S3)
    if not periodic:
        U[:, 1] = T * x
        U[:, 2] += S4 * x
        prod -= r12 * T + r13 * S4
    om = 1.7
    params = W.default_params(mode=1, n_scalars=0, Cw1=0.5, Cw2=0.73)
    F = _derive(oracle_mod, mesh, params, _stats(mesh, 0, U, (r11, r22, r33, r12, r13, r23), om))
    k = 0.5 * (r11 + r22 + r33)
    eps = k * om
    want = 0.73 - 0.5 * prod / eps
    np.testing.assert_allclose(F[:, F_SOMEGA], want, rtol=1e-12)
    # recovered gradients (the inputs of P) are the imposed ones
    np.testing.assert_allclose(F[:, 6], S, rtol=1e-12)              # d<U1>/dy
    np.testing.assert_allclose(F[:, 10], S3, rtol=1e-12)            # d<U3>/dy
    np.testing.assert_allclose(F[:, 7], 0.0 if periodic else T, atol=1e-12)   # d<U2>/dx
    # SLM G and C0 eps of R-20 from the same statistics
    np.testing.assert_allclose(F[:, F_G11], -(0.5 + 0.75 * 2.1) * om, rtol=1e-14)
    np.testing.assert_allclose(F[:, F_C0EPS], 2.1 * eps, rtol=1e-14)


# ------------------------------------------------------------ R-19 source

PAR = W.default_params()
C1, C2, G5, CV, CL, CETA = PAR["C1"], PAR["C2"], PAR["gamma5"], PAR["Cv"], PAR["CL"], PAR["Ceta"]


def _shear_case():
    stress = (0.9, 0.4, 0.6, -0.23, 0.11, 0.17)    # u11 u22 u33 u12 u13 u23
    k = 0.5 * (stress[0] + stress[1] + stress[2])
    b = {(i, j): v / (2 * k) - (1.0 / 3.0 if i == j else 0.0)
         for (i, j), v in {(0, 0): stress[0], (1, 1): stress[1], (2, 2): stress[2], (0, 1): stress[3],
                           (1, 0): stress[3], (0, 2): stress[4], (2, 0): stress[4], (1, 2): stress[5],
                           (2, 1): stress[5]}.items()}
    R = np.array([[stress[0], stress[3], stress[4]], [stress[3], stress[1], stress[5]],
                  [stress[4], stress[5], stress[2]]])
    Av = min(1.0, CV * np.linalg.det(R) / (2 * k / 3) ** 3)
    return stress, k, b, Av


def test_relaxation_source_under_simple_shear_d_U1_dy():
    """Only d<U_1>/dy = S: the source of R-19 reduces, component by
    component (derived by hand from H_ijkl), to
      r12 = k S (C2 A_v + g5/3 + g5 b11),   r21 = -k S (g5/3 + g5 b22),
      r11 = iso - k g5 b12 S,  r22 = iso + k g5 b12 S,  r33 = iso,
    with iso = (1 - C1) eps / 2."""
    import oracle
    stress, k, b, Av = _shear_case()
    S, eps = 3.0, 0.7
    r, dval, L2, av = oracle.relax_source(PAR, stress, (0, S, 0, 0, 0, 0), k, eps)
    iso = 0.5 * (1 - C1) * eps
    want = [iso - k * G5 * b[0, 1] * S,
            k * S * (C2 * Av + G5 / 3 + G5 * b[0, 0]),
            -k * S * (G5 / 3 + G5 * b[1, 1]),
            iso + k * G5 * b[0, 1] * S,
            iso]
    np.testing.assert_allclose(r, want, rtol=1e-13, atol=1e-15)
    assert av == pytest.approx(Av, rel=1e-13)
    np.testing.assert_array_equal(dval, 0.0)     # no wall normal


def test_relaxation_source_under_simple_shear_d_U2_dx_and_d_U3_dx():
    """d<U_2>/dx = T and d<U_3>/dx = S3 (the transposed shear plus an
    out-of-plane one):
      r21 = k T (C2 A_v + g5/3 + g5 b22) + k g5 b23 S3,   r12 = -k T (g5/3 + g5 b11),
      r22 = iso - k g5 b12 T,  r11 = iso + k g5 b12 T + k g5 b13 S3,
      r33 = iso - k g5 b13 S3."""
    import oracle
    stress, k, b, Av = _shear_case()
    T, S3, eps = -1.3, 2.2, 0.45
    r, _, _, _ = oracle.relax_source(PAR, stress, (0, 0, T, 0, S3, 0), k, eps)
    iso = 0.5 * (1 - C1) * eps
    want = [iso + k * G5 * b[0, 1] * T + k * G5 * b[0, 2] * S3,
            -k * T * (G5 / 3 + G5 * b[0, 0]),
            k * T * (C2 * Av + G5 / 3 + G5 * b[1, 1]) + k * G5 * b[1, 2] * S3,
            iso - k * G5 * b[0, 1] * T,
            iso - k * G5 * b[0, 2] * S3]
    np.testing.assert_allclose(r, want, rtol=1e-13, atol=1e-15)


def test_relaxation_av_limits():
    """A_v is 1 for isotropic turbulence (Cv > 1) and 0 in the
    two-component limit at a wall (<u2 u2> = 0, so det <u_i u_j> = 0)."""
    import oracle
    k, eps = 1.2, 0.8
    iso = (2 * k / 3, 2 * k / 3, 2 * k / 3, 0.0, 0.0, 0.0)
    assert oracle.relax_source(PAR, iso, (0,) * 6, k, eps)[3] == 1.0
    two = (1.4, 0.0, 1.0, 0.0, 0.0, 0.0)
    assert oracle.relax_source(PAR, two, (0,) * 6, 1.2, eps)[3] == 0.0
    # axisymmetric: <u u> = diag(3, 1, 0.5) s, k = 2.25 s: A_v = Cv 1.5 / 1.5^3
    s = 0.4
    ax = (3 * s, s, 0.5 * s, 0.0, 0.0, 0.0)
    assert oracle.relax_source(PAR, ax, (0,) * 6, 2.25 * s, eps)[3] == pytest.approx(CV * 1.5 / 1.5 ** 3, rel=1e-13)


def test_relaxation_length_scale_limits():
    """L = CL max(integral scale k^3/2 / eps, Ceta x Kolmogorov scale
    (nu^3/eps)^1/4): each branch in its own regime."""
    import oracle
    nu = 1e-3
    p = dict(PAR, nu=nu)
    iso = lambda k: (2 * k / 3, 2 * k / 3, 2 * k / 3, 0.0, 0.0, 0.0)
    # energetic turbulence: the integral scale wins
    k, eps = 2.0, 0.5
    L2 = oracle.relax_source(p, iso(k), (0,) * 6, k, eps)[2]
    assert k ** 1.5 / eps > CETA * (nu ** 3 / eps) ** 0.25
    assert math.sqrt(L2) == pytest.approx(CL * k ** 1.5 / eps, rel=1e-14)
    # near a wall, k -> 0 at finite eps: the Kolmogorov scale takes over
    k, eps = 1e-4, 5.0
    L2 = oracle.relax_source(p, iso(k), (0,) * 6, k, eps)[2]
    eta = (nu ** 3 / eps) ** 0.25
    assert CETA * eta > k ** 1.5 / eps
    assert math.sqrt(L2) == pytest.approx(CL * CETA * eta, rel=1e-14)


def test_relaxation_wall_value():
    """Wall value -4.5 eps n_i n_j: with the wall normal (0, 1) only the 22
    component is non-zero; with (1, 1)/sqrt 2 the 11, 12, 21 and 22
    components are -2.25 eps and 33 is zero."""
    import oracle
    stress, k, _, _ = _shear_case()
    eps = 0.9
    _, d, _, _ = oracle.relax_source(PAR, stress, (0,) * 6, k, eps, normal=(0.0, 1.0))
    np.testing.assert_allclose(d, [0.0, 0.0, 0.0, -4.5 * eps, 0.0], atol=1e-15)
    h = 1 / math.sqrt(2)
    _, d, _, _ = oracle.relax_source(PAR, stress, (0,) * 6, k, eps, normal=(h, h))
    np.testing.assert_allclose(d, [-2.25 * eps] * 4 + [0.0], rtol=1e-15, atol=1e-15)


def test_relaxation_uniform_periodic_box(oracle_mod):
    """Uniform statistics, no mean gradient, no walls: the relaxed tensor is
    the uniform isotropic source (1 - C1) eps / 2 delta_ij (constants solve
    (M + K_L) s = M r), so G_ij = -C1 <omega> / 2 delta_ij and
    C0 eps = 2/3 (C1 - 1) eps, whatever the anisotropy of <u_i u_j>."""
    mesh = W.unit_square(7, 0.2, periodic_x=True, periodic_y=True, seed_key=(92, 0, 0))
    params = W.default_params(mode=2, n_scalars=0)
    R = (0.5, 0.3, 0.2, 0.05, -0.04, 0.03)
    om = 2.0
    F = _derive(oracle_mod, mesh, params, _stats(mesh, 0, np.zeros((mesh.n_nodes, 3)), R, om))
    k = 0.5 * (R[0] + R[1] + R[2])
    for s in (F_G11, F_G22, F_G33):
        np.testing.assert_allclose(F[:, s], -0.5 * C1 * om, rtol=1e-9)
    np.testing.assert_allclose(F[:, F_G12], 0.0, atol=1e-9)
    np.testing.assert_allclose(F[:, F_G21], 0.0, atol=1e-9)
    np.testing.assert_allclose(F[:, F_C0EPS], (2.0 / 3.0) * (C1 - 1) * k * om, rtol=1e-9)


def test_relaxation_wall_nodes_on_a_walled_square(oracle_mod):
    """On a square with walls on all four sides, the relaxed tensor at a wall
    node is its Dirichlet value -4.5 eps n_i n_j (R-19), so with isotropic
    uniform statistics G_ij = (-4.5 eps n_i n_j - eps/2 delta_ij) / k:
    G22 = -5 <omega> on the bottom and top walls, G11 = -5 <omega> on the
    side walls, and G12 = -(+-2.25) <omega> at the corners, where the normal is
    the normalised average of the two wall normals."""
    mesh = W.unit_square(7, 0.2, periodic_x=False, periodic_y=False, seed_key=(93, 0, 0))
    params = W.default_params(mode=2, n_scalars=0)
    k, om = 0.6, 1.5
    R = (2 * k / 3, 2 * k / 3, 2 * k / 3, 0.0, 0.0, 0.0)
    F = _derive(oracle_mod, mesh, params, _stats(mesh, 0, np.zeros((mesh.n_nodes, 3)), R, om))
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    on_xw = (x == 0.0) | (x == 1.0)
    on_yw = (y == 0.0) | (y == 1.0)
    edge_y = on_yw & ~on_xw
    edge_x = on_xw & ~on_yw
    corner = on_xw & on_yw
    np.testing.assert_allclose(F[edge_y, F_G22], -5.0 * om, rtol=1e-13)
    np.testing.assert_allclose(F[edge_y, F_G11], -0.5 * om, rtol=1e-13)
    np.testing.assert_allclose(F[edge_x, F_G11], -5.0 * om, rtol=1e-13)
    np.testing.assert_allclose(F[edge_x, F_G22], -0.5 * om, rtol=1e-13)
    np.testing.assert_allclose(F[on_xw | on_yw, F_G33], -0.5 * om, rtol=1e-13)
    np.testing.assert_allclose(F[edge_x | edge_y, F_G12], 0.0, atol=1e-13)
    # corners: n1 n2 = +1/2 at (0,0) and (1,1), -1/2 at (1,0) and (0,1)
    sgn = np.where((x[corner] == y[corner]), 1.0, -1.0)
    np.testing.assert_allclose(F[corner, F_G12], -2.25 * om * sgn, rtol=1e-13)
    np.testing.assert_allclose(F[corner, F_G11], (-2.25 - 0.5) * om, rtol=1e-13)


# ------------------------------------------------------------ R-24 clamp

def test_mixing_clamp_takes_every_particle_to_its_cell_mean(oracle_mod):
    """With dt <omega> Cphi / 2 >= 1 the mixing factor is clamped at 1
    (R-24), so after one step every scalar equals its cell mean (one cell
    per element with n_bins = 1). Without the clamp the update would
    overshoot to psi - 2 (psi - m)."""
    mesh = W.unit_square(7, 0.2, periodic_x=True, periodic_y=False, seed_key=(94, 0, 0))
    dt = 1e-3
    F = W.frozen_fields(mesh, omega=2000.0, dpdx=(0.0, 0.0))
    F[:, F_G11] = F[:, F_G22] = F[:, F_G33] = 0.0
    params = W.default_params(mode=0, dt=dt, nu=0.0, n_scalars=2, n_bins=1, n_min=1, dpdx=(0.0, 0.0))
    parts = W.init_particles(mesh, 15, 2, W.rng_for(94, 0, 1), u_std=0.0)
    rng = W.rng_for(94, 0, 2)
    parts["psi"] = rng.random(parts["psi"].shape)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.fields_upload(cs, F)
    o.init()
    o.step(1)
    r = o.download(cs, len(parts["x"]))
    e = parts["elem"]
    for a in range(2):
        w = parts["weight"]
        m = np.bincount(e, w * parts["psi"][a], mesh.n_elems) / np.bincount(e, w, mesh.n_elems)
        np.testing.assert_allclose(r["psi"][a], m[e], rtol=0, atol=2e-16)


# ------------------------------------------------------------ R-20 decay

def test_slm_decay_of_k(oracle_mod):
    """Simplified Langevin model in a homogeneous periodic box with frozen
    <omega> = W (C3 = 0 and S_omega = 0 keep every particle frequency at W),
    no mean velocity gradient, viscosity or pressure gradient:
      u^{n+1} = u (1 - a W dt) + (C0 k_n W dt)^{1/2} xi,  a = 1/2 + 3/4 C0,
    so E[k^{n+1}] = k_n (1 - W dt + a^2 W^2 dt^2): k decays at the rate eps
    (dk/dt = -eps, Sec. II) up to the O(dt^2) term of forward Euler."""
    mesh = W.unit_square(4, 0.2, periodic_x=True, periodic_y=True, seed_key=(95, 0, 0))
    Wf, dt, C0 = 4.0, 0.02, 2.1
    params = W.default_params(mode=1, dt=dt, nu=0.0, n_scalars=0, dpdx=(0.0, 0.0), C0=C0, C3=0.0,
                              Cw1=0.0, Cw2=0.0, n_eff_min=0.0)
    parts = W.init_particles(mesh, 20000, 0, W.rng_for(95, 0, 1), u_std=0.5)
    parts["omega"][:] = Wf
    n = len(parts["x"])
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.init()
    a = 0.5 + 0.75 * C0
    k_of = lambda p: 0.5 * (p["u"] ** 2 + p["v"] ** 2 + p["w"] ** 2)
    k0 = np.average(k_of(parts), weights=parts["weight"])
    o.step(1)
    r = o.download(cs, n)
    kp = k_of(r)
    k1 = np.average(kp, weights=r["weight"])
    want = k0 * (1 - Wf * dt + a * a * Wf * Wf * dt * dt)
    # standard error of the weighted mean of the per-particle energies
    se = np.std(kp) / math.sqrt(n)
    assert abs(k1 - want) < 4 * se + 2e-3 * k0, (k1, want, se)
    # the O(dt^2) term matters at this dt: without it the recurrence misses
    assert abs(k1 - k0 * (1 - Wf * dt)) > 4 * se


# ------------------------------------------------------------ caps

def test_walk_cap_falls_back_to_brute_force(oracle_mod):
    """A displacement across more than 64 elements exceeds the walk cap
    (R-12): the element is then the brute-force one (R-13), the position is
    unchanged, and the fallback counter records it."""
    mesh = W.unit_square(60, 0.0, periodic_x=False, periodic_y=False, seed_key=(96, 0, 0))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=0))
    x0, y0 = 0.013, 0.51
    e0 = o.locate_brute(cs, x0, y0)
    e, x, y, u = o.walk(cs, e0, 0.987, 0.493)
    assert (x, y) == (0.987, 0.493)
    assert e == o.locate_brute(cs, x, y)
    assert o.counters(cs)["walk_fallback"] == 1
    assert o.counters(cs)["walk_steps"] == 64
    # a short walk does not fall back
    e, x, y, u = o.walk(cs, e0, 0.05, 0.52)
    assert e == o.locate_brute(cs, 0.05, 0.52)
    assert o.counters(cs)["walk_fallback"] == 1


def test_reflection_cap_falls_back(oracle_mod):
    """A point far outside a channel bounces between the two walls: after 8
    reflections (R-14) the walk stops and R-13 returns the element that
    maximises min lambda at the current (reflected) position."""
    mesh = W.unit_square(5, 0.0, periodic_x=True, periodic_y=False, seed_key=(97, 0, 0))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=0))
    e0 = o.locate_brute(cs, 0.4, 0.5)
    e, x, y, u = o.walk(cs, e0, 0.4, 20.3, (0.1, 1.0, 0.2))
    cnt = o.counters(cs)
    assert cnt["reflect"] == 8 and cnt["walk_fallback"] == 1
    # eight mirrors of y = 20.3 across y = 1 and y = 0 in turn, and the
    # velocity reversed an even number of times
    yy = 20.3
    for i in range(8):
        yy = 2.0 - yy if i % 2 == 0 else -yy
    assert y == pytest.approx(yy, abs=1e-12) and x == 0.4
    assert u == (0.1, 1.0, 0.2)
    # brute force over all elements: the largest min lambda
    info = o.mesh_info(cs)
    best, bestv = -1, -np.inf
    for q in range(mesh.n_elems):
        lam = o.bary(cs, q, x, y)
        if lam.min() > bestv:
            best, bestv = q, lam.min()
    assert e == best


def test_reflection_at_walls_of_any_orientation(oracle_mod):
    """R-14 on the polygonal walls of an annulus, whose edges face every
    direction: for each boundary edge, a point just beyond it (barycentric
    -0.1 against the edge) comes back into the same element at its mirror
    image in the edge's line, the one other point as far from both ends of
    the edge as it is, and the velocity becomes 2 u_wall - u with that
    edge's own wall velocity (each inner edge moves along itself)."""
    mesh = W.annulus(n_r=4, n_theta=24, seed_key=(98, 0, 0))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(mode=0, n_scalars=0, dpdx=(0.0, 0.0)))
    va, vb = mesh.tri[:, [1, 2, 0]], mesh.tri[:, [2, 0, 1]]
    edges = np.argwhere(mesh.edge_tag >= 0)
    assert len(edges) == 48
    u = (0.3, -0.7, 0.2)
    for e, k in edges:
        a, b = mesh.xy[va[e, k]], mesh.xy[vb[e, k]]
        mid, cen = 0.5 * (a + b), mesh.xy[mesh.tri[e]].mean(0)
        t = 1.3 * mid - 0.3 * cen
        e2, x, y, u2 = o.walk(cs, int(e), float(t[0]), float(t[1]), u)
        p = np.array([x, y])
        assert e2 == e
        assert np.linalg.norm(p - t) > 0.1 * np.linalg.norm(mid - cen)
        for q in (a, b):
            assert abs(np.linalg.norm(p - q) - np.linalg.norm(t - q)) < 1e-13
        assert o.bary(cs, int(e), x, y).min() > 0.05
        uw = np.array(mesh.bcs[mesh.edge_tag[e, k]]["u_wall"])
        np.testing.assert_allclose(u2, 2.0 * uw - np.array(u), rtol=0, atol=1e-15)
    cnt = o.counters(cs)
    assert cnt["reflect"] == len(edges) and cnt["walk_fallback"] == 0


def test_annulus_run_keeps_every_particle_inside(oracle_mod):
    """Frozen fields on the annulus (rotating inner wall), velocities of a
    tenth of the element size per step: after 30 steps every particle lies in
    the element it is assigned to, the walls have reflected particles on
    both circles, and nothing fell back or went non-finite."""
    mesh = W.annulus(n_r=4, n_theta=24, seed_key=(98, 0, 0))
    params = W.default_params(mode=0, dt=2e-3, nu=1e-3, n_scalars=0, dpdx=(0.0, 0.0))
    parts = W.init_particles(mesh, 20, 0, W.rng_for(98, 0, 1), u_std=3.0)
    F = W.frozen_fields(mesh, C0=2.1, omega=1.0, k=2.0, dpdx=(0.0, 0.0))
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.fields_upload(cs, F)
    o.init()
    o.step(30)
    n = len(parts["x"])
    r = o.download(cs, n)
    lam = np.array([o.bary(cs, int(e), x, y) for e, x, y in zip(r["elem"], r["x"], r["y"])])
    assert lam.min() > -1e-12
    rad = np.hypot(r["x"], r["y"])
    assert rad.max() <= 1.0 + 1e-12 and rad.min() >= 0.5 * math.cos(math.pi / 24) - 1e-12
    cnt = o.counters(cs)
    assert cnt["reflect"] > 50 and cnt["walk_fallback"] == 0 and cnt["nan"] == 0
    assert np.isfinite(r["u"]).all()


# ------------------------------------------------------------ regression record

def test_oracle_reproduces_its_regression_record(oracle_mod):
    """The oracle reproduces, bit for bit, the record written by
    tests/golden/make_golden.py (a guard against unintended changes of its
    arithmetic; a deliberate change regenerates the record)."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    want = np.loadtxt(mg.OUT)
    np.testing.assert_array_equal(mg.run(), want)


# ------------------------------------------------------------ R-29 / R-30 initial state

def test_initial_ensemble_distributions(oracle_mod):
    """The initial ensemble (R-29/R-30): every particle inside its element,
    its first barycentric coordinate distributed as Beta(1, 2) (the law of a
    barycentric coordinate of a point uniform in a triangle), velocity
    components N(0, u_std^2), frequency Gamma(4, scale), scalar = value
    exactly inside the disk and 0 outside, weights A_e / ppe summing to the
    domain area, ids 0..n-1 in element order."""
    from scipy import stats
    mesh = W.unit_square(6, 0.2, periodic_x=True, seed_key=(98, 0, 0))
    params = W.default_params(n_scalars=2, seed=12345, stream=3)
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    ppe, u_std, scale = 1500, 0.37, 0.21
    disk = (0.45, 0.55, 0.22, 2.5)
    n = o.particles_init(cs, ppe, u_std, scale, [disk, None])
    r = o.download(cs, n)
    assert np.array_equal(r["id"], np.arange(n, dtype=np.uint32))
    assert np.array_equal(r["elem"], np.repeat(np.arange(mesh.n_elems), ppe))
    lam = np.array([o.bary(cs, int(e), x, y) for e, x, y in zip(r["elem"][::37], r["x"][::37], r["y"][::37])])
    assert lam.min() >= -1e-15
    assert stats.kstest(lam[:, 0], lambda t: 1 - (1 - t) ** 2).pvalue > 1e-3
    assert stats.kstest(lam[:, 2], lambda t: 1 - (1 - t) ** 2).pvalue > 1e-3
    for k in ("u", "v", "w"):
        assert stats.kstest(r[k] / u_std, "norm").pvalue > 1e-3, k
    assert stats.kstest(r["omega"], stats.gamma(4, scale=scale).cdf).pvalue > 1e-3
    assert abs(np.corrcoef(r["u"], r["omega"])[0, 1]) < 4 / np.sqrt(n)
    d1, d2 = mesh.xy[mesh.tri[:, 1]] - mesh.xy[mesh.tri[:, 0]], mesh.xy[mesh.tri[:, 2]] - mesh.xy[mesh.tri[:, 0]]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    np.testing.assert_allclose(r["weight"], (area / ppe)[r["elem"]], rtol=1e-14)
    assert r["weight"].sum() == pytest.approx(1.0, rel=1e-13)
    inside = (r["x"] - disk[0]) ** 2 + (r["y"] - disk[1]) ** 2 < disk[2] ** 2
    assert np.all(r["psi"][0][inside] == disk[3]) and np.all(r["psi"][0][~inside] == 0.0)
    assert np.all(r["psi"][1] == 0.0)
    # ppe particles per element: the mass-weighted (not the counted) share of
    # the particles inside the disk is its area
    assert r["weight"][inside].sum() == pytest.approx(np.pi * disk[2] ** 2, abs=4 * np.sqrt(0.15 / n))
    # another stream gives other draws, the same stream the same ones
    o2 = oracle_mod.Oracle()
    c2 = o2.add_case(mesh, dict(params, stream=4))
    o2.particles_init(c2, ppe, u_std, scale, [disk, None])
    assert not np.array_equal(o2.download(c2, n)["u"], r["u"])
    o3 = oracle_mod.Oracle()
    c3 = o3.add_case(mesh, params)
    o3.particles_init(c3, ppe, u_std, scale, [disk, None])
    assert np.array_equal(o3.download(c3, n)["omega"], r["omega"])


def test_freezing_every_slot_is_the_frozen_field_mode(oracle_mod):
    """Mode 1 derives the fields from the statistics; with every slot frozen
    at the uploaded values it must step exactly like mode 0, which keeps the
    uploaded fields throughout. With only <omega> frozen, that slot keeps its
    value while the mean velocity slots follow the statistics."""
    mesh = W.unit_square(8, 0.2, periodic_x=True, seed_key=(6, 0, 0))
    parts = W.init_particles(mesh, 20, 1, W.rng_for(6, 0, 1), u_std=0.1, psi_disks=[(0.5, 0.5, 0.2, 1.0)])
    n = len(parts["x"])
    F = W.frozen_fields(mesh, C0=2.1, omega=1.5, k=0.01)
    runs = []
    for mode, mask in ((0, 0), (1, (1 << 22) - 1), (1, 1 << 19)):
        o = oracle_mod.Oracle()
        cs = o.add_case(mesh, W.default_params(mode=mode, n_scalars=1, dt=1e-3, nu=1e-3))
        o.fields_upload(cs, F, freeze_mask=mask)
        o.upload(cs, parts)
        o.init()
        o.step(15)
        runs.append((o.download(cs, n), o.stats(cs), o.fields(cs)))
    for k in ("x", "y", "u", "v", "w", "omega", "psi", "elem"):
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[1][2], F)
    f = runs[2][2]
    assert np.array_equal(f[:, 19], F[:, 19])
    assert not np.array_equal(f[:, 0], F[:, 0])
    with pytest.raises(RuntimeError, match="fields_upload"):
        o.fields_upload(cs, F, freeze_mask=1 << 22)


def test_rebin_variant_is_one_more_rebinning(oracle_mod):
    """R-36 (a variant of R-23): forming the bins and cell means again
    against the new fields at the end of each step. With frozen fields
    (mode 0) the new fields are the old ones, so the variant changes
    nothing, bit for bit; with fields from the statistics (mode 1) one
    variant step equals a plain step followed by an explicit rebinning."""
    mesh = W.unit_square(8, 0.2, periodic_x=True, seed_key=(6, 1, 0))
    parts = W.init_particles(mesh, 20, 1, W.rng_for(6, 1, 1), u_std=0.1, psi_disks=[(0.5, 0.5, 0.2, 1.0)])
    n = len(parts["x"])
    F = W.frozen_fields(mesh, C0=2.1, omega=1.5, k=0.01)

    def run(mode, rebin, steps, extra_rebin=False):
        o = oracle_mod.Oracle()
        cs = o.add_case(mesh, W.default_params(mode=mode, n_scalars=1, dt=1e-3, nu=1e-3, rebin=rebin))
        o.fields_upload(cs, F)
        o.upload(cs, parts)
        o.init()
        for _ in range(steps):
            o.step(1)
            if extra_rebin:
                o.rebin()
        m, cnt = o.cell_means(cs)
        return o.download(cs, n), m, cnt, o.stats(cs)

    a, b = run(0, 0, 10), run(0, 1, 10)
    for x, y in zip(a, b):
        if isinstance(x, dict):
            for k in x:
                assert np.array_equal(x[k], y[k]), k
        else:
            assert np.array_equal(x, y)
    plain, variant, explicit = run(1, 0, 3), run(1, 1, 3), run(1, 0, 3, extra_rebin=True)
    assert not np.array_equal(plain[0]["bin"], variant[0]["bin"])
    for k in ("x", "y", "u", "v", "w", "omega", "psi", "elem", "bin"):
        assert np.array_equal(variant[0][k], explicit[0][k]), k
    assert np.array_equal(variant[1], explicit[1]) and np.array_equal(variant[2], explicit[2])


# ------------------------------------------------------------ Taylor's dispersion (Sec. III.A)

def test_taylor_absolute_dispersion(oracle_mod):
    """Homogeneous frozen fields on a periodic box (SLM drift G_ii =
    -(1/2 + 3/4 C0) omega, C0 eps set for a stationary velocity variance
    sig2, uniform <U_1> = 1): every particle's cross-stream displacement
    follows the discrete Ornstein-Uhlenbeck form of Taylor's absolute
    dispersion (tests/taylor_dispersion.py), and its streamwise displacement
    has the mean <U_1> t. A wrong sign or factor in the drift, the diffusion
    C0 eps dt, the position's (2 nu dt)^{1/2} or the velocity used in Eq.(2)
    shifts the variance by more than the band; the band is three standard
    errors of a variance estimate, (2/N)^{1/2}."""
    from taylor_dispersion import discrete_variance, stationary_c0eps, taylor_variance
    mesh = W.unit_square(24, 0.2, periodic_x=True, periodic_y=True, seed_key=(5, 0, 0))
    omega, C0, dt, nu, sig2, U0 = 4.0, 2.1, 1e-3, 1e-3, 0.25, 1.0
    G = -(0.5 + 0.75 * C0) * omega
    params = W.default_params(mode=0, dt=dt, nu=nu, n_scalars=0, dpdx=(0.0, 0.0), stream=11)
    F = W.frozen_fields(mesh, C0=C0, omega=omega, dpdx=(0.0, 0.0))
    F[:, F_U1] = U0
    F[:, F_C0EPS] = stationary_c0eps(G, dt, sig2)
    parts = W.init_particles(mesh, 10, 0, W.rng_for(5, 0, 1), u_std=math.sqrt(sig2))
    parts["u"] = parts["u"] + U0
    n = len(parts["x"])
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, params)
    o.fields_upload(cs, F)
    o.upload(cs, parts)
    o.init()
    prev = o.download(cs, n)
    X = np.zeros(n)
    Y = np.zeros(n)
    done = 0
    tol = 3.0 * math.sqrt(2.0 / n)
    for check in (60, 120, 240, 360):
        while done < check:
            o.step(30)
            done += 30
            cur = o.download(cs, n)
            a, b = np.argsort(cur["id"]), np.argsort(prev["id"])
            dx = cur["x"][a] - prev["x"][b]
            dy = cur["y"][a] - prev["y"][b]
            X += dx - np.round(dx)          # unwrap the periodic shifts (box of side 1)
            Y += dy - np.round(dy)
            prev = cur
        want = discrete_variance(done, dt, G, sig2, nu)
        got = float(np.mean(Y * Y) - np.mean(Y) ** 2)
        assert abs(got / want - 1.0) < tol, (done, got, want)
        # the continuous formula is the dt -> 0 limit: O(|G| dt) apart
        t = done * dt
        assert abs(taylor_variance(t, -1.0 / G, sig2, nu) / want - 1.0) < 2.0 * abs(G) * dt
        sx = math.sqrt(float(np.var(X)) / n)
        assert abs(float(np.mean(X)) - U0 * t) < 4.0 * sx + 1e-12, (done, np.mean(X), U0 * t)
