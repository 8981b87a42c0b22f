"""Pins of the oracle's grid tables and particle tracking (Sec. I, grid roles
(i) and (iii); readings R-04, R-05, R-07, R-12..R-15, R-33).

Checked against geometry that does not go through the oracle's formulas:
barycentric coordinates at the vertices, partition of unity, Euler's formula
for the triangle count, the domain area, brute force over all elements, and
the closed forms of mirror reflection and periodic shift.
"""
import numpy as np
import pytest

import workloads as W


def _case(oracle_mod, mesh, **kw):
    o = oracle_mod.Oracle()
    cs = o.add_case(mesh, W.default_params(**kw))
    return o, cs


@pytest.fixture(scope="module")
def square(oracle_mod):
    mesh = W.unit_square(16, 0.2, periodic_x=True, periodic_y=False)
    o, cs = _case(oracle_mod, mesh)
    return mesh, o, cs


def test_barycentric_vertices_and_partition(square):
    mesh, o, cs = square
    rng = np.random.default_rng(0)
    for e in range(mesh.n_elems):
        for j in range(3):
            x, y = mesh.xy[mesh.tri[e, j]]
            lam = o.bary(cs, e, x, y)
            expect = np.eye(3)[j]
            assert np.all(np.abs(lam - expect) <= 4 * np.spacing(1.0)), (e, j, lam)
        r = rng.random(2)
        x, y = rng.random(2)
        lam = o.bary(cs, e, x, y)
        assert abs(lam.sum() - 1.0) < 1e-13
        # affine reproduction: sum lam_k x_k = x
        P = mesh.xy[mesh.tri[e]]
        assert np.allclose(lam @ P, [x, y], atol=1e-13)


def test_euler_formula_and_area(oracle_mod):
    # closed domain without periodic merge: N_e = 2 N_n - N_b - 2
    mesh = W.unit_square(12, 0.2, periodic_x=False, periodic_y=False)
    o, cs = _case(oracle_mod, mesh)
    bnodes = set()
    for e, k in zip(*np.nonzero(mesh.edge_tag >= 0)):
        bnodes.add(int(mesh.tri[e, (k + 1) % 3]))
        bnodes.add(int(mesh.tri[e, (k + 2) % 3]))
    assert mesh.n_elems == 2 * mesh.n_nodes - len(bnodes) - 2
    info = o.mesh_info(cs)
    assert info["n_stat_nodes"] == mesh.n_nodes
    assert abs(info["vol"].sum() - 1.0) < 1e-13



def test_annulus_mesh(oracle_mod):
    """The ring between two polygonal circles: Euler's formula for a domain
    with one hole (N_e = 2 N_n - N_b: no -2), the area of the ring between
    two regular n-gons, n (r1^2 - r0^2) sin(2 pi / n) / 2, 2n boundary edges
    whose ends lie on one circle, and each inner edge's wall velocity along
    the edge at spin * r0."""
    n, r0, r1 = 30, 0.4, 1.2
    mesh = W.annulus(n_r=5, n_theta=n, r0=r0, r1=r1, spin=2.0, seed_key=(95, 0, 0))
    o, cs = _case(oracle_mod, mesh)
    edges = np.argwhere(mesh.edge_tag >= 0)
    assert len(edges) == 2 * n
    bnodes = set()
    for e, k in edges:
        a, b = mesh.xy[mesh.tri[e, (k + 1) % 3]], mesh.xy[mesh.tri[e, (k + 2) % 3]]
        bnodes.update((int(mesh.tri[e, (k + 1) % 3]), int(mesh.tri[e, (k + 2) % 3])))
        ra, rb = np.hypot(*a), np.hypot(*b)
        assert abs(ra - rb) < 1e-12 and min(abs(ra - r0), abs(ra - r1)) < 1e-12
        uw = np.array(mesh.bcs[mesh.edge_tag[e, k]]["u_wall"][:2])
        if abs(ra - r0) < 1e-12:
            t = (b - a) / np.linalg.norm(b - a)
            assert abs(abs(uw @ t) - 2.0 * r0) < 1e-12 and abs(uw @ np.array([-t[1], t[0]])) < 1e-12
        else:
            assert not uw.any()
    assert mesh.n_elems == 2 * mesh.n_nodes - len(bnodes)
    area = 0.5 * n * (r1 ** 2 - r0 ** 2) * np.sin(2 * np.pi / n)
    assert abs(o.mesh_info(cs)["vol"].sum() - area) < 1e-13 * area

def test_periodic_merge(square):
    mesh, o, cs = square
    info = o.mesh_info(cs)
    # the right column (x = 1) are images of the left column
    right = np.nonzero(mesh.xy[:, 0] == 1.0)[0]
    left = np.nonzero(mesh.xy[:, 0] == 0.0)[0]
    assert info["n_stat_nodes"] == mesh.n_nodes - right.size
    sn = info["stat_node"]
    for r in right:
        l = left[np.nonzero(mesh.xy[left, 1] == mesh.xy[r, 1])[0][0]]
        assert sn[r] == sn[l]
    # lumped areas of merged nodes sum to the domain area
    uniq = np.unique(sn, return_index=True)[1]
    assert abs(info["vol"][uniq].sum() - 1.0) < 1e-13


def test_channel_mesh_periodic_partners(oracle_mod):
    mesh = W.channel(n_half=10, nx=20)
    o, cs = _case(oracle_mod, mesh, mode=2)
    info = o.mesh_info(cs)
    ncol = np.sum(mesh.xy[:, 0] == 0.0)
    assert info["n_stat_nodes"] == mesh.n_nodes - ncol
    uniq = np.unique(info["stat_node"], return_index=True)[1]
    assert abs(info["vol"][uniq].sum() - 2 * 2 * np.pi) < 1e-11


def test_mesh_rejections(oracle_mod):
    mesh = W.unit_square(6, 0.0, periodic_x=True)
    bad = W.Mesh("cw", mesh.xy, mesh.tri[:, [0, 2, 1]].copy(), mesh.edge_tag, mesh.bcs)
    with pytest.raises(RuntimeError, match="counter-clockwise"):
        _case(oracle_mod, bad)
    # periodic partner missing: shift the right boundary
    bcs = [dict(b) for b in mesh.bcs]
    bcs[2] = dict(type=W.BC_PERIODIC, shift=(0.5, 0.0))
    with pytest.raises(RuntimeError, match="partner"):
        _case(oracle_mod, W.Mesh("p", mesh.xy, mesh.tri, mesh.edge_tag, bcs))
    # interior edge carrying a boundary tag
    tag = mesh.edge_tag.copy()
    e, k = next((e, k) for e in range(mesh.n_elems) for k in range(3) if tag[e, k] < 0)
    tag[e, k] = 0
    with pytest.raises(RuntimeError, match="interior edge|orientation"):
        _case(oracle_mod, W.Mesh("t", mesh.xy, mesh.tri, tag, mesh.bcs))


def test_walk_against_brute_force(square):
    mesh, o, cs = square
    rng = np.random.default_rng(3)
    for _ in range(3000):
        x, y = rng.random(2)
        e0 = int(rng.integers(mesh.n_elems))
        e, xn, yn, _ = o.walk(cs, e0, x, y)
        assert (xn, yn) == (x, y)
        lam = o.bary(cs, e, x, y)
        assert lam.min() >= 0.0
        b = o.locate_brute(cs, x, y)
        lb = o.bary(cs, b, x, y)
        # unique containing element when the point is away from every edge
        if min(lam.min(), lb.min()) > 1e-12:
            assert e == b


def test_walk_adversarial_points(square):
    mesh, o, cs = square
    pts = []
    for e in range(0, mesh.n_elems, 7):
        P = mesh.xy[mesh.tri[e]]
        pts += [P[0], 0.5 * (P[0] + P[1]), 0.5 * (P[1] + P[2]), P.mean(0)]
    rng = np.random.default_rng(4)
    for x, y in pts:
        if not (0.0 < y < 1.0):
            continue
        e0 = int(rng.integers(mesh.n_elems))
        e, xn, yn, _ = o.walk(cs, e0, float(x), float(y))
        lam = o.bary(cs, e, xn, yn)
        assert lam.min() >= -1e-14


def test_wall_reflection_closed_form(square, oracle_mod):
    mesh, o, cs = square
    # find an element touching the bottom wall y = 0
    e = next(e for e in range(mesh.n_elems) if (mesh.edge_tag[e] == 0).any())
    P = mesh.xy[mesh.tri[e]]
    cx = float(P[:, 0].mean())
    x, y = cx, -0.0123
    e2, xn, yn, u = o.walk(cs, e, x, y, (0.3, -0.7, 0.2))
    assert xn == x and yn == 0.0123
    assert u == (-0.3, 0.7, -0.2)
    assert o.bary(cs, e2, xn, yn).min() >= 0.0
    # the lid: U <- 2 U_w - U
    lidmesh = W.unit_square(8, 0.2, periodic_x=True, lid=(1.0, 0.0, 0.0))
    o2, cs2 = _case(oracle_mod, lidmesh)
    e = next(e for e in range(lidmesh.n_elems) if (lidmesh.edge_tag[e] == 1).any())
    cx = float(lidmesh.xy[lidmesh.tri[e]][:, 0].mean())
    e2, xn, yn, u = o2.walk(cs2, e, cx, 1.01, (0.25, 0.5, 0.0))
    assert yn == pytest.approx(0.99, abs=1e-15)
    assert u == (1.75, -0.5, 0.0)


def test_periodic_shift_closed_form(square):
    mesh, o, cs = square
    e = next(e for e in range(mesh.n_elems) if (mesh.edge_tag[e] == 3).any())
    y = float(mesh.xy[mesh.tri[e]][:, 1].mean())
    e2, xn, yn, u = o.walk(cs, e, 1.0 + 0.03125, y, (1.0, 0.0, 0.0))
    assert xn == 0.03125 and yn == y and u == (1.0, 0.0, 0.0)
    assert o.bary(cs, e2, xn, yn).min() >= 0.0
    e3, xn, yn, _ = o.walk(cs, e2, -0.25, y)
    assert xn == 0.75
    assert o.bary(cs, e3, xn, yn).min() >= 0.0
    c = o.counters(cs)
    assert c["periodic"] >= 2
