"""FP64 CPU oracle of the particle advance (test infrastructure).

Plain, slow, single-threaded C (``oracle/*.c``) wrapped with ctypes. Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark load it;
the GPU library never does, and the two share no source. What it computes is
stated in ``oracle.h`` and in the C files, each step citing the paper's
equation (Eq.(2), (4), (5), (6), (9)) or section, and the reading (R-nn) that
fixes what the paper leaves open.

Pins that are not yet tied to anything but the oracle itself: the coupled
full model over many steps (elliptic relaxation + projection) is
"parity unpinned" beyond agreement with the GPU path -- the paper prints no
numbers for it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SOURCES = ["orc_api.c", "orc_fem.c", "orc_locate.c", "orc_mesh.c", "orc_model.c", "orc_rng.c"]

NF = 22
NCOUNT = 12
COUNTER_NAMES = ["walk_fallback", "reflect", "periodic", "omega_flip", "empty_node", "nan",
                 "walk_steps", "cg_iters_er", "cg_iters_p", "cg_fail", "k_floor", "eps_floor"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES]
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", _LIB_PATH + ".tmp"] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _BC(C.Structure):
    _fields_ = [("type", C.c_int32), ("u_wall", C.c_double * 3), ("shift", C.c_double * 2)]


class _Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("n_elems", C.c_int32), ("tri", C.POINTER(C.c_int32)),
                ("edge_tag", C.POINTER(C.c_int32)),
                ("n_bc", C.c_int32), ("bc", C.POINTER(_BC))]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("dt", C.c_double), ("nu", C.c_double),
                ("C0", C.c_double), ("C3", C.c_double), ("C4", C.c_double),
                ("Cw1", C.c_double), ("Cw2", C.c_double), ("Cphi", C.c_double),
                ("C1", C.c_double), ("C2", C.c_double), ("gamma5", C.c_double),
                ("Cv", C.c_double), ("CL", C.c_double), ("Ceta", C.c_double),
                ("dpdx", C.c_double * 2),
                ("n_scalars", C.c_int32), ("n_bins", C.c_int32), ("n_min", C.c_int32),
                ("src", (C.c_double * 4) * 4),
                ("k_floor", C.c_double), ("eps_floor", C.c_double),
                ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
                ("seed", C.c_uint64), ("stream", C.c_uint32), ("n_eff_min", C.c_double),
                ("reaction", C.c_int32), ("k_react", C.c_double * 4), ("rebin", C.c_int32)]


class _InitParams(C.Structure):
    _fields_ = [("u_std", C.c_double), ("omega_scale", C.c_double), ("disk", (C.c_double * 4) * 4)]


def init_params_struct(u_std, omega_scale, disks=()):
    ip = _InitParams()
    ip.u_std, ip.omega_scale = float(u_std), float(omega_scale)
    for a, dk in enumerate(disks):
        if dk is None:
            continue
        for j in range(4):
            ip.disk[a][j] = float(dk[j])
    return ip


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.POINTER(C.c_double)) for k in
                                     ("x", "y", "u", "v", "w", "omega", "weight", "psi")] + \
               [("elem", C.POINTER(C.c_int32)), ("id", C.POINTER(C.c_uint32)),
                ("bin", C.POINTER(C.c_uint8))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_last_error.restype = C.c_char_p
        L.orc_last_error.argtypes = [C.c_void_p]
        L.orc_ln.restype = C.c_double
        L.orc_ln.argtypes = [C.c_double]
        L.orc_sincos2pi.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_gauss6.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_double)]
        L.orc_uniform6.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_double)]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_locate_brute.restype = C.c_int32
        L.orc_locate_brute.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double]
        L.orc_walk.restype = C.c_int32
        L.orc_walk.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_set_step_index.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_fem_helmholtz.argtypes = [C.c_void_p, C.c_int32] + [C.c_void_p] * 4 + [C.c_double, C.c_void_p]
        L.orc_fem_projection.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                         C.c_double, C.c_void_p]
        for name in ("orc_add_case", "orc_mesh_info", "orc_particles_upload", "orc_particles_download",
                     "orc_fields_upload", "orc_fields_download", "orc_pressure_download", "orc_pressure_upload", "orc_init",
                     "orc_rebin", "orc_step", "orc_stats", "orc_node_sums", "orc_cell_means",
                     "orc_counters", "orc_bary", "orc_recover", "orc_set_stats", "orc_derive",
                     "orc_particles_init"):
            getattr(L, name).restype = C.c_int
        L.orc_relax_source.restype = C.c_int
        L.orc_relax_source.argtypes = [C.c_void_p] + [C.POINTER(C.c_double)] * 2 + [C.c_double, C.c_double] + \
            [C.POINTER(C.c_double)] * 5
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# ---------------------------------------------------------------- primitives

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def ln(u: float) -> float:
    return lib().orc_ln(float(u))


def sincos2pi(u: float):
    s, c = C.c_double(), C.c_double()
    lib().orc_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def gauss6(seed, pid, step, stream):
    o = (C.c_double * 6)()
    lib().orc_gauss6(seed, pid, step, stream, o)
    return np.array(o[:])


def relax_source(params, stress, grad, k, eps, normal=(0.0, 0.0)):
    """Elliptic-relaxation source of R-19 at one node: stress = <u1u1>,
    <u2u2>, <u3u3>, <u1u2>, <u1u3>, <u2u3>; grad = d<U_i>/dx_j (i-major,
    j = x, y). Returns (r, dval) for the components 11, 12, 21, 22, 33, L^2
    and A_v."""
    ps = _params_struct(params)
    st = (C.c_double * 6)(*[float(v) for v in stress])
    gr = (C.c_double * 6)(*[float(v) for v in grad])
    nn = (C.c_double * 2)(*[float(v) for v in normal])
    r, dv = (C.c_double * 5)(), (C.c_double * 5)()
    L2, Av = C.c_double(), C.c_double()
    rc = lib().orc_relax_source(C.byref(ps), st, gr, float(k), float(eps), nn, r, dv, C.byref(L2), C.byref(Av))
    if rc != 0:
        raise RuntimeError("orc_relax_source failed")
    return np.array(r[:]), np.array(dv[:]), L2.value, Av.value


def uniform6(seed, pid, step, stream):
    o = (C.c_double * 6)()
    lib().orc_uniform6(seed, pid, step, stream, o)
    return np.array(o[:])


# ---------------------------------------------------------------- context

def _mesh_struct(mesh):
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64).reshape(-1)
    tri = np.ascontiguousarray(mesh.tri, dtype=np.int32).reshape(-1)
    tag = np.ascontiguousarray(mesh.edge_tag, dtype=np.int32).reshape(-1)
    bcs = (_BC * max(1, len(mesh.bcs)))()
    for i, b in enumerate(mesh.bcs):
        bcs[i].type = int(b["type"])
        for j in range(3):
            bcs[i].u_wall[j] = float(b.get("u_wall", (0, 0, 0))[j])
        for j in range(2):
            bcs[i].shift[j] = float(b.get("shift", (0, 0))[j])
    m = _Mesh(mesh.n_nodes, _dp(xy), mesh.n_elems, _ip(tri), _ip(tag), len(mesh.bcs), bcs)
    return m, (xy, tri, tag, bcs)


def _params_struct(p):
    s = _Params()
    for name, _ in _Params._fields_:
        if name in ("dpdx", "src", "reaction", "k_react", "rebin"):
            continue
        setattr(s, name, p[name])
    s.dpdx[0], s.dpdx[1] = p["dpdx"]
    s.reaction = int(p.get("reaction", 0))
    s.rebin = int(p.get("rebin", 0))
    kr = list(p.get("k_react", ()))
    for a in range(4):
        s.k_react[a] = float(kr[a]) if a < len(kr) else 0.0
    src = np.zeros((4, 4))
    if len(p.get("src", [])):
        src[:len(p["src"])] = np.asarray(p["src"], dtype=np.float64)
    for a in range(4):
        for j in range(4):
            s.src[a][j] = src[a, j]
    return s


class Oracle:
    """Host-memory twin of the GPU library's call sequence."""

    def __init__(self):
        self._L = lib()
        self._c = C.c_void_p(self._L.orc_create())
        self._cases = []

    def __del__(self):
        try:
            if self._c:
                self._L.orc_destroy(self._c)
                self._c = None
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"oracle {what}: {self._L.orc_last_error(self._c).decode()} (code {rc})")

    def add_case(self, mesh, params):
        m, keep = _mesh_struct(mesh)
        ps = _params_struct(params)
        cid = C.c_int32()
        self._check(self._L.orc_add_case(self._c, C.byref(m), C.byref(ps), C.byref(cid)), "add_case")
        self._cases.append((mesh, dict(params)))
        return cid.value

    def mesh_info(self, cs):
        mesh = self._cases[cs][0]
        nsn = C.c_int32()
        snode = np.zeros(mesh.n_nodes, np.int32)
        nbr = np.zeros(3 * mesh.n_elems, np.int32)
        rec = np.zeros(8 * mesh.n_elems)
        vol = np.zeros(mesh.n_nodes)
        self._check(self._L.orc_mesh_info(self._c, cs, C.byref(nsn), _ip(snode), _ip(nbr), _dp(rec), _dp(vol)),
                    "mesh_info")
        return dict(n_stat_nodes=nsn.value, stat_node=snode, nbr=nbr.reshape(-1, 3),
                    rec=rec.reshape(-1, 8), vol=vol)

    def upload(self, cs, parts):
        n = len(parts["x"])
        ns = self._cases[cs][1]["n_scalars"]
        arrs = {k: np.ascontiguousarray(parts[k], dtype=np.float64) for k in
                ("x", "y", "u", "v", "w", "omega", "weight")}
        psi = np.ascontiguousarray(parts["psi"], dtype=np.float64).reshape(-1) if ns else np.zeros(1)
        elem = np.ascontiguousarray(parts["elem"], dtype=np.int32)
        pid = np.ascontiguousarray(parts["id"], dtype=np.uint32)
        b = np.ascontiguousarray(parts.get("bin", np.zeros(n, np.uint8)), dtype=np.uint8)
        st = _Particles(n, *[_dp(arrs[k]) for k in ("x", "y", "u", "v", "w", "omega", "weight")], _dp(psi),
                        _ip(elem), pid.ctypes.data_as(C.POINTER(C.c_uint32)),
                        b.ctypes.data_as(C.POINTER(C.c_uint8)))
        self._check(self._L.orc_particles_upload(self._c, cs, C.byref(st)), "upload")

    def particles_init(self, cs, ppe, u_std=0.1, omega_scale=0.25, disks=()):
        """Initial ensemble of R-29/R-30 (ppe particles per element, drawn from
        the case's generator with purpose 1); returns the particle count."""
        ip = init_params_struct(u_std, omega_scale, disks)
        self._check(self._L.orc_particles_init(self._c, cs, int(ppe), C.byref(ip)), "particles_init")
        return self._cases[cs][0].n_elems * int(ppe)

    def download(self, cs, n):
        ns = self._cases[cs][1]["n_scalars"]
        out = {k: np.zeros(n) for k in ("x", "y", "u", "v", "w", "omega", "weight")}
        psi = np.zeros(max(1, ns * n))
        elem = np.zeros(n, np.int32)
        pid = np.zeros(n, np.uint32)
        b = np.zeros(n, np.uint8)
        st = _Particles(n, *[_dp(out[k]) for k in ("x", "y", "u", "v", "w", "omega", "weight")], _dp(psi),
                        _ip(elem), pid.ctypes.data_as(C.POINTER(C.c_uint32)),
                        b.ctypes.data_as(C.POINTER(C.c_uint8)))
        self._check(self._L.orc_particles_download(self._c, cs, C.byref(st)), "download")
        out["psi"] = psi[:ns * n].reshape(ns, n)
        out["elem"], out["id"], out["bin"] = elem, pid, b
        return out

    def fields_upload(self, cs, F, freeze_mask=0):
        F = np.ascontiguousarray(F, dtype=np.float64)
        self._check(self._L.orc_fields_upload(self._c, cs, _dp(F), C.c_uint32(int(freeze_mask))), "fields_upload")

    def pressure_upload(self, cs, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        self._check(self._L.orc_pressure_upload(self._c, cs, _dp(P)), "pressure_upload")

    def fields(self, cs):
        mesh = self._cases[cs][0]
        F = np.zeros((mesh.n_nodes, NF))
        self._check(self._L.orc_fields_download(self._c, cs, _dp(F)), "fields_download")
        return F

    def pressure(self, cs):
        mesh = self._cases[cs][0]
        P = np.zeros(mesh.n_nodes)
        self._check(self._L.orc_pressure_download(self._c, cs, _dp(P)), "pressure")
        return P

    def init(self):
        self._check(self._L.orc_init(self._c), "init")

    def rebin(self):
        self._check(self._L.orc_rebin(self._c), "rebin")

    def set_step_index(self, n):
        self._check(self._L.orc_set_step_index(self._c, n), "set_step_index")

    def step(self, n=1):
        self._check(self._L.orc_step(self._c, n), "step")

    def stats(self, cs):
        mesh, p = self._cases[cs]
        out = np.zeros((mesh.n_nodes, 12 + 2 * p["n_scalars"]))
        self._check(self._L.orc_stats(self._c, cs, _dp(out)), "stats")
        return out

    def node_sums(self, cs):
        mesh, p = self._cases[cs]
        out = np.zeros((mesh.n_nodes, 12 + 2 * p["n_scalars"]))
        self._check(self._L.orc_node_sums(self._c, cs, _dp(out)), "node_sums")
        return out

    def cell_means(self, cs):
        mesh, p = self._cases[cs]
        ns = p["n_scalars"]
        mean = np.zeros(max(1, mesh.n_elems * 8 * ns))
        cnt = np.zeros(mesh.n_elems * 8, np.int32)
        self._check(self._L.orc_cell_means(self._c, cs, _dp(mean), _ip(cnt)), "cell_means")
        return mean[:mesh.n_elems * 8 * ns].reshape(mesh.n_elems, 8, ns), cnt.reshape(mesh.n_elems, 8)

    def counters(self, cs):
        out = np.zeros(NCOUNT, np.int64)
        self._check(self._L.orc_counters(self._c, cs, out.ctypes.data_as(C.POINTER(C.c_int64))), "counters")
        return dict(zip(COUNTER_NAMES, out.tolist()))

    def set_stats(self, cs, stats):
        """Overwrite the node statistics (per raw node, the layout of stats())."""
        st = np.ascontiguousarray(stats, dtype=np.float64)
        self._check(self._L.orc_set_stats(self._c, cs, _dp(st)), "set_stats")

    def derive(self, cs, project=False):
        """Eulerian fields from the current node statistics (and the
        projection when `project`)."""
        self._check(self._L.orc_derive(self._c, cs, int(bool(project))), "derive")

    def bary(self, cs, e, x, y):
        lam = (C.c_double * 3)()
        self._check(self._L.orc_bary(self._c, cs, e, C.c_double(x), C.c_double(y), lam), "bary")
        return np.array(lam[:])

    def locate_brute(self, cs, x, y):
        return self._L.orc_locate_brute(self._c, cs, x, y)

    def walk(self, cs, e0, x, y, u3=(0.0, 0.0, 0.0)):
        cx, cy = C.c_double(x), C.c_double(y)
        cu = (C.c_double * 3)(*u3)
        e = self._L.orc_walk(self._c, cs, e0, C.byref(cx), C.byref(cy), cu)
        return e, cx.value, cy.value, tuple(cu[:])

    def recover(self, cs, f):
        mesh = self._cases[cs][0]
        f = np.ascontiguousarray(f, dtype=np.float64)
        gx, gy, lap = np.zeros(mesh.n_nodes), np.zeros(mesh.n_nodes), np.zeros(mesh.n_nodes)
        self._check(self._L.orc_recover(self._c, cs, _dp(f), _dp(gx), _dp(gy), _dp(lap)), "recover")
        return gx, gy, lap

    def helmholtz(self, cs, L2, r, dmask, dval, tol=1e-13):
        mesh = self._cases[cs][0]
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (L2, r, dval)]
        dm = np.ascontiguousarray(dmask, dtype=np.int32)
        s = np.zeros(mesh.n_nodes)
        self._check(self._L.orc_fem_helmholtz(self._c, cs, a[0].ctypes.data, a[1].ctypes.data,
                                              dm.ctypes.data, a[2].ctypes.data, tol, s.ctypes.data),
                    "helmholtz")
        return s

    def projection(self, cs, U1, U2, dt, tol=1e-13):
        mesh = self._cases[cs][0]
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (U1, U2)]
        phi = np.zeros(mesh.n_nodes)
        self._check(self._L.orc_fem_projection(self._c, cs, a[0].ctypes.data, a[1].ctypes.data,
                                               dt, tol, phi.ctypes.data), "projection")
        return phi
