"""Pins of the oracle's Eulerian side: gradient recovery (R-16), the Galerkin
elliptic-relaxation solve (R-19) and the pressure projection (R-27), i.e.
the grid's role (ii) in Sec. I, plus the Reynolds-stress trace identity that
fixes C0 eps from G_ij (Eq.(4) must dissipate k at the rate eps, Sec. II).

Pins: exactness for linear fields, manufactured solutions converging at
second order on refined meshes, the L = 0 limit, divergence-free input giving
zero pressure correction.
"""
import math

import numpy as np
import pytest

import workloads as W


def _oracle_case(oracle_mod, mesh, **kw):
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(**kw))
    return o, cs


def test_recovery_exact_for_linear_fields(oracle_mod):
    mesh = W.unit_square(14, 0.25, periodic_x=False, periodic_y=False)
    o, cs = _oracle_case(oracle_mod, mesh)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    f = 0.3 + 1.7 * x - 2.2 * y
    gx, gy, lap = o.recover(cs, f)
    assert np.allclose(gx, 1.7, atol=1e-12)
    assert np.allclose(gy, -2.2, atol=1e-12)
    assert np.abs(lap).max() < 1e-10


def test_recovery_laplacian_of_quadratic(oracle_mod):
    errs = []
    for n in (9, 17, 33):
        mesh = W.unit_square(n, 0.0, periodic_x=False, periodic_y=False)
        o, cs = _oracle_case(oracle_mod, mesh)
        x, y = mesh.xy[:, 0], mesh.xy[:, 1]
        gx, gy, lap = o.recover(cs, x * x + 3 * y * y)
        inner = (x > 0.2) & (x < 0.8) & (y > 0.2) & (y < 0.8)
        assert np.allclose(gx[inner], 2 * x[inner], atol=1e-10)
        errs.append(np.abs(lap[inner] - 8.0).max())
    # on the uniform split grid the recovered Laplacian is exact in the interior
    assert max(errs) < 1e-8


def _periodic_square(n):
    return W.unit_square(n, 0.0, periodic_x=True, periodic_y=True)


def test_helmholtz_L0_reproduces_rhs(oracle_mod):
    mesh = W.unit_square(12, 0.2, periodic_x=True, periodic_y=True)
    o, cs = _oracle_case(oracle_mod, mesh)
    rng = np.random.default_rng(1)
    info = o.mesh_info(cs)
    r = rng.standard_normal(info["n_stat_nodes"])[info["stat_node"]]
    s = o.helmholtz(cs, np.zeros(mesh.n_nodes), r, np.zeros(mesh.n_nodes, np.int32), np.zeros(mesh.n_nodes))
    assert np.allclose(s, r, atol=1e-11)


@pytest.mark.parametrize("walls", [False, True])
def test_helmholtz_manufactured_second_order(oracle_mod, walls):
    c = 0.01
    errs, hs = [], []
    for n in (9, 17, 33):
        mesh = W.unit_square(n, 0.0, periodic_x=True, periodic_y=not walls)
        o, cs = _oracle_case(oracle_mod, mesh)
        x, y = mesh.xy[:, 0], mesh.xy[:, 1]
        if walls:
            ex = np.sin(np.pi * y) * np.cos(2 * np.pi * x)
            lapfac = np.pi ** 2 + 4 * np.pi ** 2
        else:
            ex = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
            lapfac = 8 * np.pi ** 2
        r = (1 + c * lapfac) * ex
        dmask = ((y == 0.0) | (y == 1.0)).astype(np.int32) if walls else np.zeros(mesh.n_nodes, np.int32)
        s = o.helmholtz(cs, np.full(mesh.n_nodes, c), r, dmask, np.zeros(mesh.n_nodes))
        errs.append(np.abs(s - ex).max())
        hs.append(1.0 / (n - 1))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(slopes > 1.8), (errs, slopes)


def test_projection_zero_for_uniform_flow(oracle_mod):
    mesh = W.channel(n_half=8, nx=24)
    o, cs = _oracle_case(oracle_mod, mesh, mode=2)
    phi = o.projection(cs, np.full(mesh.n_nodes, 1.3), np.zeros(mesh.n_nodes), 1e-3)
    assert np.abs(phi).max() < 1e-9


def test_projection_manufactured_second_order(oracle_mod):
    errs, hs = [], []
    dt = 0.01
    for n in (9, 17, 33):
        mesh = _periodic_square(n)
        o, cs = _oracle_case(oracle_mod, mesh)
        x, y = mesh.xy[:, 0], mesh.xy[:, 1]
        psi = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) / (2 * np.pi)
        U1 = np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)     # d psi / dx
        U2 = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)     # d psi / dy
        phi = o.projection(cs, U1, U2, dt)
        ex = psi / dt
        info = o.mesh_info(cs)
        rows = np.unique(info["stat_node"], return_index=True)[1]
        ex = ex - ex[rows].mean()
        errs.append(np.abs(phi - ex).max() * dt)
        hs.append(1.0 / (n - 1))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(slopes > 1.8), (errs, slopes)


def _trace_identity(F, st):
    # 2 G_ik <u_i u_k> + 3 C0 eps = -2 eps  (k budget of Eq.(4): dk/dt = -eps)
    u11, u22, u33, u12 = st[:, 5], st[:, 6], st[:, 7], st[:, 8]
    GR = F[:, 14] * u11 + F[:, 15] * u12 + F[:, 16] * u12 + F[:, 17] * u22 + F[:, 18] * u33
    k = 0.5 * (u11 + u22 + u33)
    eps = k * st[:, 11]
    return 2 * GR + 3 * F[:, 20], -2 * eps


@pytest.mark.parametrize("mode", [1, 2])
def test_reynolds_stress_trace_identity(oracle_mod, mode):
    if mode == 1:
        cfg = W.config_small()
    else:
        mesh = W.channel(n_half=10, nx=24)
        params = W.default_params(mode=2, dt=5e-4, nu=1 / 1080, n_scalars=1)
        cfg = dict(mesh=mesh, params=params,
                   particles=W.init_particles(mesh, 40, 1, np.random.default_rng(3), u_std=1.0))
    o = oracle_mod.Oracle()
    cs = o.add_case(cfg["mesh"], cfg["params"])
    o.upload(cs, cfg["particles"])
    o.init()
    F, st = o.fields(cs), o.stats(cs)
    lhs, rhs = _trace_identity(F, st)
    ok = F[:, 20] > 0           # where C0 eps is not clipped at zero
    assert ok.mean() > 0.5
    assert np.allclose(lhs[ok], rhs[ok], rtol=1e-9, atol=1e-12)
    if mode == 2:
        # wall nodes carry the Dirichlet value: G_12 = wp_12/k = 0 for walls y = const
        y = cfg["mesh"].xy[:, 1]
        wall = (y == 0.0) | (y == 2.0)
        assert np.abs(F[wall, 15]).max() < 1e-12 and np.abs(F[wall, 16]).max() < 1e-12
