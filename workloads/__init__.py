"""Seeded synthetic inputs: meshes, initial particle ensembles and case settings.

This module holds no arithmetic of the method. It produces *inputs* that the
FP64 oracle and the GPU library both consume: triangle meshes shaped like the
paper's two test cases (the channel of Sec. III.A, the cavity of Sec. III.B),
the unit square used as a small parity case, initial particle states (the
recipes of readings R-29/R-30) and the model constants (R-19, R-20, R-22).

Everything is derived from numpy ``SeedSequence`` streams spawned from the
project seed, so every run sees the same inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PROJECT_SEED = 10060549

BC_WALL = 0
BC_PERIODIC = 1


@dataclasses.dataclass
class Mesh:
    name: str
    xy: np.ndarray        # (n_nodes, 2) float64
    tri: np.ndarray       # (n_elems, 3) int32, counter-clockwise
    edge_tag: np.ndarray  # (n_elems, 3) int32, edge k opposite vertex k; -1 interior
    bcs: list             # dicts: type, u_wall, shift

    @property
    def n_nodes(self):
        return int(self.xy.shape[0])

    @property
    def n_elems(self):
        return int(self.tri.shape[0])


def rng_for(*keys) -> np.random.Generator:
    """Generator for a (config, case, purpose) key path below the project seed."""
    ss = np.random.SeedSequence([PROJECT_SEED] + [int(k) for k in keys])
    return np.random.default_rng(ss)


# ----------------------------------------------------------------- meshes

def _orient_ccw(xy, tri):
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    d = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    tri = tri.copy()
    flip = d < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def _tag_edges(xy, tri, classify):
    """Tag the boundary edges (edges used by one triangle) with classify(pa, pb)."""
    ne = tri.shape[0]
    tag = np.full((ne, 3), -1, np.int32)
    a = tri[:, [1, 2, 0]].reshape(-1)
    b = tri[:, [2, 0, 1]].reshape(-1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo.astype(np.int64) * (xy.shape[0] + 1) + hi
    uniq, cnt = np.unique(key, return_counts=True)
    once = set(uniq[cnt == 1].tolist())
    for i in range(3 * ne):
        if int(key[i]) in once:
            t = classify(xy[a[i]], xy[b[i]])
            if t < 0:
                raise ValueError(f"boundary edge {xy[a[i]]}-{xy[b[i]]} not on any boundary")
            tag[i // 3, i % 3] = t
    return tag


def _delaunay(points):
    from scipy.spatial import Delaunay
    d = Delaunay(points)
    tri = d.simplices.astype(np.int32)
    tri = _orient_ccw(points, tri)
    a, b, c = points[tri[:, 0]], points[tri[:, 1]], points[tri[:, 2]]
    area = 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))
    keep = area > 0
    used = np.zeros(points.shape[0], bool)
    used[tri[keep].reshape(-1)] = True
    if not keep.all() or not used.all():
        raise ValueError("Delaunay produced degenerate triangles or unused points")
    return tri


def _rect_classifier(x0, x1, y0, y1, tags):
    """tags = (bottom, top, left, right) boundary indices."""
    def classify(pa, pb):
        if pa[1] == y0 and pb[1] == y0:
            return tags[0]
        if pa[1] == y1 and pb[1] == y1:
            return tags[1]
        if pa[0] == x0 and pb[0] == x0:
            return tags[2]
        if pa[0] == x1 and pb[0] == x1:
            return tags[3]
        return -1
    return classify


def unit_square(n: int = 16, jitter: float = 0.2, periodic_x: bool = True, periodic_y: bool = False,
                lid=None, seed_key=(0, 0, 0)) -> Mesh:
    """n x n nodes on [0,1]^2, interior nodes jittered by U(-jitter h, jitter h),
    each cell split along its (i,j)-(i+1,j+1) diagonal: 2(n-1)^2 triangles.
    Boundaries: 0 bottom, 1 top, 2 left, 3 right."""
    h = 1.0 / (n - 1)
    rng = rng_for(*seed_key)
    xs = np.arange(n) * h
    X, Y = np.meshgrid(xs, xs, indexing="ij")   # X[i,j] = i h
    X[-1, :] = 1.0
    Y[:, -1] = 1.0
    jx = rng.uniform(-jitter * h, jitter * h, size=(n, n))
    jy = rng.uniform(-jitter * h, jitter * h, size=(n, n))
    inner = np.zeros((n, n), bool)
    inner[1:-1, 1:-1] = True
    X = np.where(inner, X + jx, X)
    Y = np.where(inner, Y + jy, Y)
    xy = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)

    def nid(i, j):
        return i * n + j
    tris = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    tri = _orient_ccw(xy, np.array(tris, np.int32))
    tag = _tag_edges(xy, tri, _rect_classifier(0.0, 1.0, 0.0, 1.0, (0, 1, 2, 3)))
    lidv = (0.0, 0.0, 0.0) if lid is None else tuple(lid)
    if periodic_y:
        b0 = dict(type=BC_PERIODIC, shift=(0.0, 1.0))
        b1 = dict(type=BC_PERIODIC, shift=(0.0, -1.0))
    else:
        b0 = dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0))
        b1 = dict(type=BC_WALL, u_wall=lidv)
    if periodic_x:
        b2 = dict(type=BC_PERIODIC, shift=(1.0, 0.0))
        b3 = dict(type=BC_PERIODIC, shift=(-1.0, 0.0))
    else:
        b2 = dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0))
        b3 = dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0))
    return Mesh(f"square{n}", xy, tri, tag, [b0, b1, b2, b3])


def _geometric_levels(first: float, n: int, length: float) -> np.ndarray:
    """n + 1 levels from 0 to length, spacings first * r^i with r solved so the
    spacings sum to length."""
    if first * n >= length:
        return np.linspace(0.0, length, n + 1)
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        r = 0.5 * (lo + hi)
        s = first * (r ** n - 1.0) / (r - 1.0)
        if s > length:
            hi = r
        else:
            lo = r
    r = 0.5 * (lo + hi)
    sp = first * r ** np.arange(n)
    lev = np.concatenate([[0.0], np.cumsum(sp)])
    lev *= length / lev[-1]
    lev[-1] = length
    return lev


def channel(n_half: int = 48, nx: int = 105, first: float = 1e-3, Lx: float = 2 * math.pi, H: float = 2.0,
            seed_key=(1, 0, 0)) -> Mesh:
    """Channel [0,Lx] x [0,H], periodic in x, walls at y = 0 and y = H.
    y-levels graded geometrically from both walls (first spacing `first`,
    n_half levels to the centreline); nx points per level with x-jitter
    +-0.3 dx, interior levels jittered +-0.2 of the local y-spacing; the two
    periodic columns carry identical y values. Delaunay triangulation.
    Boundaries: 0 bottom wall, 1 top wall, 2 left (shift +Lx), 3 right (shift -Lx)."""
    rng = rng_for(*seed_key)
    half = _geometric_levels(first, n_half, 0.5 * H)
    ys = np.concatenate([half, H - half[-2::-1]])
    nl = ys.size
    dy_lo = np.diff(ys, prepend=np.nan)
    dy_hi = np.diff(ys, append=np.nan)
    dx = Lx / nx
    pts = []
    for j in range(nl):
        y = ys[j]
        if 0 < j < nl - 1:
            y = y + rng.uniform(-0.2, 0.2) * min(dy_lo[j], dy_hi[j])
        pts.append((0.0, y))
        pts.append((Lx, y))
        xi = (np.arange(1, nx) + rng.uniform(-0.3, 0.3, size=nx - 1)) * dx
        for x in xi:
            pts.append((float(x), y))
    xy = np.array(pts, np.float64)
    xy[xy[:, 1] == 0.0, 1] = 0.0
    tri = _delaunay(xy)
    tag = _tag_edges(xy, tri, _rect_classifier(0.0, Lx, 0.0, H, (0, 1, 2, 3)))
    bcs = [dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0)), dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0)),
           dict(type=BC_PERIODIC, shift=(Lx, 0.0)), dict(type=BC_PERIODIC, shift=(-Lx, 0.0))]
    return Mesh(f"channel{tri.shape[0]}", xy, tri, tag, bcs)


def cavity(n_half: int = 112, first: float = 1e-3, lid: float = 1.0, seed_key=(3, 0, 0),
           regularized: bool = True) -> Mesh:
    """Unit-square cavity with walls everywhere, the top one moving at `lid`.
    Tensor levels graded geometrically from every wall (n_half levels to the
    middle), interior points jittered +-0.2 of the local spacing. Delaunay.
    Boundaries: 0 bottom, 1 top (lid), 2 left, 3 right. With `regularized`,
    every lid edge carries a wall of its own moving at lid * 16 x^2 (1-x)^2
    (x at the edge midpoint): the lid speed then falls to zero at the two top
    corners instead of jumping there, which removes the corner singularity of
    the mean pressure."""
    rng = rng_for(*seed_key)
    half = _geometric_levels(first, n_half, 0.5)
    lev = np.concatenate([half, 1.0 - half[-2::-1]])
    n = lev.size
    d_lo = np.diff(lev, prepend=np.nan)
    d_hi = np.diff(lev, append=np.nan)
    loc = np.minimum(d_lo, d_hi)
    X, Y = np.meshgrid(lev, lev, indexing="ij")
    jx = rng.uniform(-0.2, 0.2, size=(n, n)) * loc[:, None]
    jy = rng.uniform(-0.2, 0.2, size=(n, n)) * loc[None, :]
    inner = np.zeros((n, n), bool)
    inner[1:-1, 1:-1] = True
    X = np.where(inner, X + jx, X)
    Y = np.where(inner, Y + jy, Y)
    xy = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    tri = _delaunay(xy)
    tag = _tag_edges(xy, tri, _rect_classifier(0.0, 1.0, 0.0, 1.0, (0, 1, 2, 3)))
    bcs = [dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0)), dict(type=BC_WALL, u_wall=(lid, 0.0, 0.0)),
           dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0)), dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0))]
    if regularized:
        va, vb = tri[:, [1, 2, 0]], tri[:, [2, 0, 1]]
        for e, k in np.argwhere(tag == 1):
            xm = 0.5 * (xy[va[e, k], 0] + xy[vb[e, k], 0])
            tag[e, k] = len(bcs)
            bcs.append(dict(type=BC_WALL, u_wall=(lid * 16.0 * xm * xm * (1.0 - xm) ** 2, 0.0, 0.0)))
    return Mesh(f"cavity{tri.shape[0]}", xy, tri, tag, bcs)


def annulus(n_r: int = 8, n_theta: int = 50, r0: float = 0.5, r1: float = 1.0, spin: float = 1.0,
            jitter: float = 0.2, seed_key=(6, 0, 0)) -> Mesh:
    """Ring r0 <= r <= r1 between two circular walls drawn as polygons: n_theta
    nodes on each circle at the angles 2 pi j / n_theta, n_r radial intervals,
    interior nodes jittered by +-jitter of the local spacing in r and theta;
    each quadrilateral cell split along one diagonal, alternating. The outer
    wall is at rest. Every edge of the inner wall is a wall of its own moving
    at spin * r0 along the edge (the circle's tangent at the edge's mid-angle,
    counter-clockwise): a rotating inner cylinder. Boundaries: 0 the outer
    wall, 1..n_theta the inner wall's edges."""
    rng = rng_for(*seed_key)
    dr, dth = (r1 - r0) / n_r, 2.0 * math.pi / n_theta
    r = r0 + dr * np.arange(n_r + 1)[:, None] + np.zeros((1, n_theta))
    th = dth * np.arange(n_theta)[None, :] + np.zeros((n_r + 1, 1))
    r[1:-1] += rng.uniform(-jitter, jitter, size=(n_r - 1, n_theta)) * dr
    th[1:-1] += rng.uniform(-jitter, jitter, size=(n_r - 1, n_theta)) * dth
    xy = np.stack([(r * np.cos(th)).reshape(-1), (r * np.sin(th)).reshape(-1)], axis=1)
    tri = []
    for i in range(n_r):
        for j in range(n_theta):
            a, b = i * n_theta + j, i * n_theta + (j + 1) % n_theta
            c, d = b + n_theta, a + n_theta
            tri += [(a, b, c), (a, c, d)] if (i + j) % 2 == 0 else [(a, b, d), (b, c, d)]
    tri = _orient_ccw(xy, np.array(tri, np.int32))
    if not (element_areas(Mesh("", xy, tri, None, [])) > 0).all():
        raise ValueError("annulus: degenerate triangle")

    def classify(pa, pb):
        ra, rb = math.hypot(*pa), math.hypot(*pb)
        if abs(ra - r1) < 1e-12 and abs(rb - r1) < 1e-12:
            return 0
        if abs(ra - r0) < 1e-12 and abs(rb - r0) < 1e-12:
            return 1
        return -1

    tag = _tag_edges(xy, tri, classify)
    bcs = [dict(type=BC_WALL, u_wall=(0.0, 0.0, 0.0))]
    va, vb = tri[:, [1, 2, 0]], tri[:, [2, 0, 1]]
    for e, k in np.argwhere(tag == 1):
        m = 0.5 * (xy[va[e, k]] + xy[vb[e, k]])
        t = np.array([-m[1], m[0]]) / math.hypot(*m)
        tag[e, k] = len(bcs)
        bcs.append(dict(type=BC_WALL, u_wall=(spin * r0 * t[0], spin * r0 * t[1], 0.0)))
    return Mesh(f"annulus{tri.shape[0]}", xy, tri, tag, bcs)


# ----------------------------------------------------------------- particles

def element_areas(mesh: Mesh) -> np.ndarray:
    a, b, c = (mesh.xy[mesh.tri[:, k]] for k in range(3))
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))


def init_particles(mesh: Mesh, ppe: int, n_scalars: int, rng: np.random.Generator, *,
                   u_std: float = 0.1, omega_shape: float = 4.0, omega_scale: float = 0.25,
                   psi_disks=(), equal_mass: bool = False) -> dict:
    """ne * ppe particles, uniform within each element (R-29), velocities
    N(0, u_std^2) per component, frequency Gamma(omega_shape, omega_scale),
    scalar alpha = value inside its initial disk (cx, cy, r, value) else 0,
    id = index (R-32). Mass weights (R-31): ppe particles per element of
    weight area / ppe, or with equal_mass the same total count spread in
    proportion to element area (largest remainders), every particle weighing
    total area / count."""
    ne = mesh.n_elems
    n = ne * ppe
    if equal_mass:
        area = element_areas(mesh)
        share = area / area.sum() * n
        cnt = np.floor(share).astype(np.int64)
        rest = n - int(cnt.sum())
        if rest > 0:
            cnt[np.argsort(-(share - cnt), kind="stable")[:rest]] += 1
        elem = np.repeat(np.arange(ne, dtype=np.int32), cnt)
    else:
        elem = np.repeat(np.arange(ne, dtype=np.int32), ppe)
    r1 = rng.random(n)
    r2 = rng.random(n)
    s1 = np.sqrt(r1)
    lam = np.stack([1.0 - s1, s1 * (1.0 - r2), s1 * r2], axis=1)
    P = mesh.xy[mesh.tri[elem]]            # (n, 3, 2)
    xy = np.einsum("nk,nkd->nd", lam, P)
    u = rng.normal(0.0, u_std, size=(3, n))
    om = rng.gamma(omega_shape, omega_scale, size=n)
    psi = np.zeros((n_scalars, n))
    for a, disk in enumerate(psi_disks):
        if a >= n_scalars or disk is None:
            continue
        cx, cy, r, val = disk
        inside = (xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2 < r * r
        psi[a, inside] = val
    if equal_mass:
        weight = np.full(n, element_areas(mesh).sum() / n)
    else:
        weight = (element_areas(mesh) / ppe)[elem]
    return dict(x=xy[:, 0].copy(), y=xy[:, 1].copy(), u=u[0].copy(), v=u[1].copy(), w=u[2].copy(),
                omega=om, weight=weight, psi=psi, elem=elem, id=np.arange(n, dtype=np.uint32),
                bin=np.zeros(n, np.uint8))


# ----------------------------------------------------------------- settings

def default_params(**over) -> dict:
    """Model constants (R-19, R-20, R-22, R-24) and numerical settings."""
    p = dict(mode=1, dt=1e-3, nu=1e-3,
             C0=2.1, C3=1.0, C4=0.25, Cw1=0.5, Cw2=0.73, Cphi=2.0,
             C1=1.85, C2=0.63, gamma5=0.1, Cv=1.4, CL=0.134, Ceta=72.0,
             dpdx=(-1.0, 0.0), n_scalars=1, n_bins=8, n_min=4, src=[],
             k_floor=1e-12, eps_floor=1e-12, cg_rtol=1e-10, cg_maxit=2000,
             seed=PROJECT_SEED, stream=0, n_eff_min=8.0, reaction=0, k_react=(0.0, 0.0, 0.0, 0.0),
             rebin=0)
    p.update(over)
    return p


def frozen_fields(mesh: Mesh, *, C0=2.1, omega=1.0, k=None, dpdx=(-1.0, 0.0)) -> np.ndarray:
    """Uniform nodal fields for frozen-field tests: zero mean velocity and
    gradients, pressure gradient dpdx, SLM G_ij = -(1/2 + 3/4 C0) omega
    delta_ij, C0 eps = C0 k omega when k is given (else 0)."""
    F = np.zeros((mesh.n_nodes, 22))
    F[:, 3], F[:, 4] = dpdx
    g = -(0.5 + 0.75 * C0) * omega
    F[:, 14] = F[:, 17] = F[:, 18] = g
    F[:, 19] = omega
    F[:, 20] = 0.0 if k is None else C0 * k * omega
    return F


# ----------------------------------------------------------------- configurations

def config_small(seed_key=(0,)):
    """Unit square, 16x16 nodes (450 triangles), 50 particles per element,
    periodic in x, walls in y; velocities N(0, 0.01), frequency Gamma(4, 1/4),
    one scalar = 1 inside the disk of radius 0.1 at the centre; frozen mean
    pressure gradient (-1, 0) and simplified Langevin G_ij; dt = 1e-3."""
    mesh = unit_square(16, 0.2, periodic_x=True, periodic_y=False, seed_key=(0, 0, 0))
    params = default_params(mode=1, dt=1e-3, nu=1e-3, n_scalars=1, dpdx=(-1.0, 0.0), stream=0)
    parts = init_particles(mesh, 50, 1, rng_for(0, 0, 1), u_std=0.1,
                           psi_disks=[(0.5, 0.5, 0.1, 1.0)])
    return dict(name="square450-fp64", mesh=mesh, params=params, particles=parts, steps=100)


def config_channel(ppe: int = 100, n_half: int = 48, nx: int = 105):
    """Channel [0,2pi] x [0,2] at Re_tau = 1080 (nu = 1/1080, driving mean
    pressure gradient -1), ~20k triangles graded to the walls (first cell
    1e-3), 100 particles per element, one scalar released continuously from
    a disk of radius 0.02 at (1.0, 0.5); full model (elliptic relaxation +
    projection); velocities N(0,1), frequency Gamma(4, 1/4); dt = 5e-4."""
    mesh = channel(n_half=n_half, nx=nx, seed_key=(1, 0, 0))
    params = default_params(mode=2, dt=5e-4, nu=1.0 / 1080.0, n_scalars=1, dpdx=(-1.0, 0.0),
                            src=[(1.0, 0.5, 0.02, 1.0)], stream=1)
    parts = init_particles(mesh, ppe, 1, rng_for(1, 0, 1), u_std=1.0)
    return dict(name=f"channel{mesh.n_elems}", mesh=mesh, params=params, particles=parts, steps=1000)


def config_cavity(ppe: int = 100, n_half: int = 112):
    """Lid-driven cavity on the unit square at Re = 4000 (nu = 1/4000, lid
    speed 1), ~100k triangles refined at all walls, 100 particles per
    element, two scalars from disks of radius 0.02 at (0.25, 0.1) and
    (0.75, 0.1); velocities N(0, 0.01), frequency Gamma(4, 1/4); dt = 2e-4."""
    mesh = cavity(n_half=n_half, seed_key=(3, 0, 0))
    params = default_params(mode=2, dt=2e-4, nu=1.0 / 4000.0, n_scalars=2, dpdx=(0.0, 0.0),
                            src=[(0.25, 0.1, 0.02, 1.0), (0.75, 0.1, 0.02, 1.0)], stream=3)
    parts = init_particles(mesh, ppe, 2, rng_for(3, 0, 1), u_std=0.1)
    return dict(name=f"cavity{mesh.n_elems}", mesh=mesh, params=params, particles=parts, steps=500)


def config_batched(n_cases: int = 32, ne_range=(2000, 50000), ppe_range=(50, 200), seed_key=(4,),
                   dt_channel=(2e-4, 1e-3), dt_cavity=(1e-4, 3e-4)):
    """Batch of independent flows advanced together: shapes alternate channel /
    cavity, element counts log-uniform in ne_range (level counts scaled by
    sqrt(N_e)), particles per element uniform integer in ppe_range, 0..4
    scalars released from disks of radius 0.02 whose centres keep 0.1 from the
    walls, time step log-uniform in dt_channel or dt_cavity (the explicit
    Euler steps of the cavity's lid shear layer need the smaller range to stay
    stable over a few hundred steps); full model."""
    rng = rng_for(*seed_key, 0)
    cases = []
    for c in range(n_cases):
        ne_t = float(np.exp(rng.uniform(np.log(ne_range[0]), np.log(ne_range[1]))))
        ppe = int(rng.integers(ppe_range[0], ppe_range[1] + 1))
        ns = int(rng.integers(0, 5))
        udt = rng.uniform(0.0, 1.0)
        kind = "channel" if c % 2 == 0 else "cavity"
        lo, hi = dt_channel if kind == "channel" else dt_cavity
        dt = float(np.exp(np.log(lo) + udt * (np.log(hi) - np.log(lo))))
        if kind == "channel":
            s = np.sqrt(ne_t / 20160.0)
            mesh = channel(n_half=max(4, int(round(48 * s))), nx=max(8, int(round(105 * s))), seed_key=(4, c, 0))
            Lx, H, ustd, nu, dpdx = 2 * np.pi, 2.0, 1.0, 1.0 / 1080.0, (-1.0, 0.0)
        else:
            s = np.sqrt(ne_t / 100352.0)
            mesh = cavity(n_half=max(6, int(round(112 * s))), seed_key=(4, c, 0))
            Lx, H, ustd, nu, dpdx = 1.0, 1.0, 0.1, 1.0 / 4000.0, (0.0, 0.0)
        src = [(float(rng.uniform(0.1, Lx - 0.1)), float(rng.uniform(0.1, H - 0.1)), 0.02, 1.0) for _ in range(ns)]
        params = default_params(mode=2, dt=dt, nu=nu, n_scalars=ns, dpdx=dpdx, src=src, stream=100 + c)
        parts = init_particles(mesh, ppe, ns, rng_for(4, c, 1), u_std=ustd)
        cases.append(dict(name=f"{kind}{mesh.n_elems}", mesh=mesh, params=params, particles=parts, ppe=ppe))
    return dict(name=f"batch{n_cases}", cases=cases, steps=100)
