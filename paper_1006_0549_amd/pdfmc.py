"""Python binding of libpdfmc.so (argument marshalling only).

Every step of the particle advance runs in the HIP kernels behind the C ABI
declared in include/pdfmc.h; this module only converts arguments. PyTorch
provides the device workspace (one uint8 tensor) and the HIP stream. If the
library has not been built, or no GPU is visible, the calls raise -- there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdfmc.so")

FP64, FP32 = 0, 1
NF = 22
N_COUNTERS = 13
COUNTER_NAMES = ["walk_fallback", "reflect", "periodic", "omega_flip", "empty_node", "nan",
                 "walk_steps", "cg_iters_er", "cg_iters_p", "cg_fail", "k_floor", "eps_floor",
                 "scatter_overflow"]
STATUS = {0: "OK", 1: "INVALID", 2: "MESH", 3: "NOMEM", 4: "HIP", 5: "STATE", 6: "UNSUPPORTED"}


class PdfmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pdfmc {STATUS.get(code, code)}: {msg}")
        self.code = code


class _BC(C.Structure):
    _fields_ = [("type", C.c_int32), ("u_wall", C.c_double * 3), ("shift", C.c_double * 2)]


class _MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("xy", C.c_void_p), ("n_elems", C.c_int32), ("tri", C.c_void_p),
                ("edge_tag", C.c_void_p), ("n_bc", C.c_int32), ("bc", C.POINTER(_BC))]


class _CaseParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("dt", C.c_double), ("nu", C.c_double),
                ("C0", C.c_double), ("C3", C.c_double), ("C4", C.c_double), ("Cw1", C.c_double),
                ("Cw2", C.c_double), ("Cphi", C.c_double), ("C1", C.c_double), ("C2", C.c_double),
                ("gamma5", C.c_double), ("Cv", C.c_double), ("CL", C.c_double), ("Ceta", C.c_double),
                ("dpdx", C.c_double * 2), ("n_scalars", C.c_int32), ("n_bins", C.c_int32),
                ("n_min", C.c_int32), ("src", (C.c_double * 4) * 4), ("k_floor", C.c_double),
                ("eps_floor", C.c_double), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32),
                ("seed", C.c_uint64), ("stream", C.c_uint32), ("n_eff_min", C.c_double),
                ("reaction", C.c_int32), ("k_react", C.c_double * 4), ("rebin", C.c_int32)]


class _TuneResult(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("sort_interval", C.c_int32), ("tail_rows", C.c_int32),
                ("trials", C.c_int32), ("steps", C.c_int32), ("ms_per_step", C.c_double)]


class _InitParams(C.Structure):
    _fields_ = [("u_std", C.c_double), ("omega_scale", C.c_double), ("disk", (C.c_double * 4) * 4)]


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in
                                     ("x", "y", "u", "v", "w", "omega", "weight", "psi", "elem", "id", "bin")]


_lib = None
EXPORTS = ["pdfmc_create", "pdfmc_destroy", "pdfmc_last_error", "pdfmc_add_case", "pdfmc_case_info",
           "pdfmc_workspace_query", "pdfmc_workspace_bind", "pdfmc_particles_upload", "pdfmc_particles_init",
           "pdfmc_particles_download", "pdfmc_fields_upload", "pdfmc_fields_download",
           "pdfmc_pressure_download", "pdfmc_init", "pdfmc_rebin", "pdfmc_step", "pdfmc_set_step_index",
           "pdfmc_stats_readback", "pdfmc_node_sums", "pdfmc_cell_means", "pdfmc_counters",
           "pdfmc_set_options", "pdfmc_sort", "pdfmc_sort_noalloc", "pdfmc_synchronize", "pdfmc_timing", "pdfmc_timing_read",
           "pdfmc_draw_gaussians", "pdfmc_set_solver", "pdfmc_solver_info", "pdfmc_autotune",
           "pdfmc_set_projection_solver", "pdfmc_projection_info"]


def lib():
    """Load libpdfmc.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.pdfmc_create.argtypes = [C.POINTER(vp), C.c_int32, vp]
        L.pdfmc_destroy.argtypes = [vp]
        L.pdfmc_destroy.restype = None
        L.pdfmc_last_error.argtypes = [vp]
        L.pdfmc_last_error.restype = C.c_char_p
        L.pdfmc_add_case.argtypes = [vp, C.POINTER(_MeshDesc), C.POINTER(_CaseParams), C.c_int64,
                                     C.POINTER(C.c_int32)]
        L.pdfmc_case_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), vp]
        L.pdfmc_workspace_query.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.pdfmc_workspace_bind.argtypes = [vp, vp, C.c_uint64]
        L.pdfmc_particles_upload.argtypes = [vp, C.c_int32, C.POINTER(_Particles)]
        L.pdfmc_particles_init.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(_InitParams)]
        L.pdfmc_particles_download.argtypes = [vp, C.c_int32, C.POINTER(_Particles)]
        L.pdfmc_fields_upload.argtypes = [vp, C.c_int32, vp, C.c_uint32]
        for f in ("pdfmc_fields_download", "pdfmc_pressure_download",
                  "pdfmc_stats_readback", "pdfmc_node_sums", "pdfmc_counters"):
            getattr(L, f).argtypes = [vp, C.c_int32, vp]
        L.pdfmc_cell_means.argtypes = [vp, C.c_int32, vp, vp]
        for f in ("pdfmc_init", "pdfmc_rebin", "pdfmc_sort", "pdfmc_sort_noalloc", "pdfmc_synchronize"):
            getattr(L, f).argtypes = [vp]
        L.pdfmc_step.argtypes = [vp, C.c_int32, C.c_uint32]
        L.pdfmc_set_step_index.argtypes = [vp, C.c_uint32]
        L.pdfmc_set_options.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.pdfmc_timing.argtypes = [vp, C.c_int32]
        L.pdfmc_set_solver.argtypes = [vp, C.c_int32, C.c_int32]
        L.pdfmc_autotune.argtypes = [vp, C.c_int32, C.POINTER(_TuneResult)]
        L.pdfmc_solver_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.pdfmc_set_projection_solver.argtypes = [vp, C.c_int32]
        L.pdfmc_projection_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.pdfmc_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.pdfmc_draw_gaussians.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, C.c_int64, vp]
        for f in EXPORTS:
            if f not in ("pdfmc_destroy", "pdfmc_last_error"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


class Sim:
    """One library context on the current torch stream of `device`."""

    def __init__(self, precision: str = "fp64", device: str = "cuda:0", stream=None, host_only: bool = False):
        """host_only=True gives a context for the host-side calls only (mesh
        validation, workspace size); it cannot bind a workspace."""
        import torch
        self.torch = torch
        self.host_only = host_only
        self.prec = FP64 if precision == "fp64" else FP32
        self.precision = precision
        handle = None
        if not host_only:
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible: the pdfmc library runs on the GPU only")
            self.device = torch.device(device)
            # a stream of our own (default priority): graph capture needs a
            # stream other than the legacy default stream
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            handle = self.stream.cuda_stream
        self._L = lib()
        h = C.c_void_p()
        self._check(self._L.pdfmc_create(C.byref(h), self.prec, C.c_void_p(handle)), "create", ctx=False)
        self._h = h
        self._cases = []
        self._ws = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._L.pdfmc_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _check(self, rc, what, ctx=True):
        if rc != 0:
            msg = self._L.pdfmc_last_error(self._h).decode() if ctx else ""
            raise PdfmcError(rc, f"{what}: {msg}")

    # ------------------------------------------------------------ setup
    def add_case(self, mesh, params, capacity: int) -> int:
        xy = np.ascontiguousarray(mesh.xy, np.float64)
        tri = np.ascontiguousarray(mesh.tri, np.int32)
        tag = np.ascontiguousarray(mesh.edge_tag, np.int32)
        bcs = (_BC * max(1, len(mesh.bcs)))()
        for i, b in enumerate(mesh.bcs):
            bcs[i].type = int(b["type"])
            for j in range(3):
                bcs[i].u_wall[j] = float(b.get("u_wall", (0.0, 0.0, 0.0))[j])
            for j in range(2):
                bcs[i].shift[j] = float(b.get("shift", (0.0, 0.0))[j])
        md = _MeshDesc(mesh.n_nodes, xy.ctypes.data, mesh.n_elems, tri.ctypes.data, tag.ctypes.data,
                       len(mesh.bcs), bcs)
        p = _CaseParams()
        for name, _ in _CaseParams._fields_:
            if name not in ("dpdx", "src", "reaction", "k_react", "rebin"):
                setattr(p, name, params[name])
        p.dpdx[0], p.dpdx[1] = params["dpdx"]
        p.reaction = int(params.get("reaction", 0))
        p.rebin = int(params.get("rebin", 0))
        kr = list(params.get("k_react", ()))
        for a in range(4):
            p.k_react[a] = float(kr[a]) if a < len(kr) else 0.0
        for a, s in enumerate(params.get("src", [])):
            for j in range(4):
                p.src[a][j] = float(s[j])
        cid = C.c_int32()
        self._check(self._L.pdfmc_add_case(self._h, C.byref(md), C.byref(p), int(capacity), C.byref(cid)), "add_case")
        self._cases.append((mesh, dict(params), int(capacity)))
        return cid.value

    def case_info(self, cs):
        mesh = self._cases[cs][0]
        n = C.c_int32()
        sn = np.zeros(mesh.n_nodes, np.int32)
        self._check(self._L.pdfmc_case_info(self._h, cs, C.byref(n), sn.ctypes.data), "case_info")
        return n.value, sn

    def workspace_bytes(self) -> int:
        b = C.c_uint64()
        self._check(self._L.pdfmc_workspace_query(self._h, C.byref(b)), "workspace_query")
        return b.value

    def bind(self):
        if self.host_only:
            raise RuntimeError("a host-only context cannot bind a device workspace")
        nbytes = self.workspace_bytes()
        with self.torch.cuda.stream(self.stream):
            self._ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        self._check(self._L.pdfmc_workspace_bind(self._h, C.c_void_p(self._ws.data_ptr()), nbytes), "workspace_bind")
        return nbytes

    def set_options(self, sort_interval=0, block_size=256, use_graph=False):
        self._check(self._L.pdfmc_set_options(self._h, sort_interval, block_size, int(bool(use_graph))), "set_options")

    def set_solver(self, iterations=0, tail_rows=64):
        """iterations = 0: adaptive number of row-parallel CG iterations."""
        self._check(self._L.pdfmc_set_solver(self._h, int(iterations), int(tail_rows)), "set_solver")

    def autotune(self, steps_per_trial=4):
        """Pick block size, sort interval and multigrid tail threshold by timing
        real steps (the trial steps advance the simulation)."""
        r = _TuneResult()
        self._check(self._L.pdfmc_autotune(self._h, int(steps_per_trial), C.byref(r)), "autotune")
        return dict(block_size=r.block_size, sort_interval=r.sort_interval, tail_rows=r.tail_rows,
                    trials=r.trials, steps=r.steps, ms_per_step=r.ms_per_step)

    def solver_info(self):
        it, lv = C.c_int32(), C.c_int32()
        self._check(self._L.pdfmc_solver_info(self._h, C.byref(it), C.byref(lv)), "solver_info")
        return it.value, lv.value

    PROJECTION_METHODS = {"direct": 0, "pcg": 1}

    def set_projection_solver(self, method="direct"):
        """"direct": sweeps over the Cholesky factor of the constant projection
        matrix; "pcg": the multigrid PCG of the relaxation."""
        if method not in self.PROJECTION_METHODS:
            raise ValueError(f"projection method must be one of {list(self.PROJECTION_METHODS)}")
        self._check(self._L.pdfmc_set_projection_solver(self._h, self.PROJECTION_METHODS[method]),
                    "set_projection_solver")

    def projection_info(self):
        m, h, v = C.c_int32(), C.c_int32(), C.c_int64()
        self._check(self._L.pdfmc_projection_info(self._h, C.byref(m), C.byref(h), C.byref(v)), "projection_info")
        return dict(method="direct" if m.value == 0 else "pcg", height=h.value, factor_values=v.value)

    # ------------------------------------------------------------ particles and fields
    def upload(self, cs, parts):
        ns = self._cases[cs][1]["n_scalars"]
        n = len(parts["x"])
        keep = {k: np.ascontiguousarray(parts[k], np.float64) for k in ("x", "y", "u", "v", "w", "omega", "weight")}
        keep["psi"] = np.ascontiguousarray(parts["psi"], np.float64).reshape(-1) if ns else None
        keep["elem"] = np.ascontiguousarray(parts["elem"], np.int32)
        keep["id"] = np.ascontiguousarray(parts["id"], np.uint32)
        keep["bin"] = np.ascontiguousarray(parts["bin"], np.uint8) if "bin" in parts else None
        st = _Particles(n, *[_ptr(keep[k]) for k in ("x", "y", "u", "v", "w", "omega", "weight", "psi",
                                                     "elem", "id", "bin")])
        self._check(self._L.pdfmc_particles_upload(self._h, cs, C.byref(st)), "particles_upload")

    def init_particles(self, cs, ppe, u_std=0.1, omega_scale=0.25, disks=()):
        """Draw the initial ensemble on the device (ppe particles per element;
        disks[a] = (cx, cy, r, value) for scalar a); returns the particle count."""
        ip = _InitParams()
        ip.u_std, ip.omega_scale = float(u_std), float(omega_scale)
        for a, dk in enumerate(disks):
            if dk is not None:
                for j in range(4):
                    ip.disk[a][j] = float(dk[j])
        self._check(self._L.pdfmc_particles_init(self._h, cs, int(ppe), C.byref(ip)), "particles_init")
        return self._cases[cs][0].n_elems * int(ppe)

    def download(self, cs, n):
        ns = self._cases[cs][1]["n_scalars"]
        out = {k: np.zeros(n) for k in ("x", "y", "u", "v", "w", "omega", "weight")}
        out["psi"] = np.zeros((ns, n))
        out["elem"] = np.zeros(n, np.int32)
        out["id"] = np.zeros(n, np.uint32)
        out["bin"] = np.zeros(n, np.uint8)
        st = _Particles(n, *[_ptr(out[k]) for k in ("x", "y", "u", "v", "w", "omega", "weight")],
                        _ptr(out["psi"]) if ns else None, _ptr(out["elem"]), _ptr(out["id"]), _ptr(out["bin"]))
        self._check(self._L.pdfmc_particles_download(self._h, cs, C.byref(st)), "particles_download")
        return out

    def fields_upload(self, cs, F, freeze_mask=0):
        """Fields per raw node; bit q of freeze_mask keeps slot q at these
        values in every later step."""
        F = np.ascontiguousarray(F, np.float64)
        self._check(self._L.pdfmc_fields_upload(self._h, cs, F.ctypes.data, int(freeze_mask)), "fields_upload")

    def fields(self, cs):
        F = np.zeros((self._cases[cs][0].n_nodes, NF))
        self._check(self._L.pdfmc_fields_download(self._h, cs, F.ctypes.data), "fields_download")
        return F

    def pressure(self, cs):
        P = np.zeros(self._cases[cs][0].n_nodes)
        self._check(self._L.pdfmc_pressure_download(self._h, cs, P.ctypes.data), "pressure_download")
        return P

    # ------------------------------------------------------------ stepping
    def init(self):
        self._check(self._L.pdfmc_init(self._h), "init")

    def rebin(self):
        self._check(self._L.pdfmc_rebin(self._h), "rebin")

    STAGE_ADVANCE, STAGE_STATS, STAGE_FIELDS, STAGE_ALL = 1, 2, 4, 7

    def step(self, n=1, stages=7):
        self._check(self._L.pdfmc_step(self._h, int(n), int(stages)), "step")

    def set_step_index(self, n):
        self._check(self._L.pdfmc_set_step_index(self._h, int(n)), "set_step_index")

    def sort(self):
        self._check(self._L.pdfmc_sort(self._h), "sort")

    def sort_noalloc(self):
        """The sort with static device scratch (asynchronous, allocates nothing)."""
        self._check(self._L.pdfmc_sort_noalloc(self._h), "sort_noalloc")

    def synchronize(self):
        self._check(self._L.pdfmc_synchronize(self._h), "synchronize")

    # ------------------------------------------------------------ readback
    def stats(self, cs):
        mesh, p, _ = self._cases[cs]
        out = np.zeros((mesh.n_nodes, 12 + 2 * p["n_scalars"]))
        self._check(self._L.pdfmc_stats_readback(self._h, cs, out.ctypes.data), "stats_readback")
        return out

    def node_sums(self, cs):
        mesh, p, _ = self._cases[cs]
        out = np.zeros((mesh.n_nodes, 12 + 2 * p["n_scalars"]))
        self._check(self._L.pdfmc_node_sums(self._h, cs, out.ctypes.data), "node_sums")
        return out

    def cell_means(self, cs):
        mesh, p, _ = self._cases[cs]
        ns = p["n_scalars"]
        mean = np.zeros(max(1, mesh.n_elems * 8 * ns))
        cnt = np.zeros(mesh.n_elems * 8, np.int32)
        self._check(self._L.pdfmc_cell_means(self._h, cs, mean.ctypes.data, cnt.ctypes.data), "cell_means")
        return mean[:mesh.n_elems * 8 * ns].reshape(mesh.n_elems, 8, ns), cnt.reshape(mesh.n_elems, 8)

    def counters(self, cs):
        out = np.zeros(N_COUNTERS, np.int64)
        self._check(self._L.pdfmc_counters(self._h, cs, out.ctypes.data), "counters")
        return dict(zip(COUNTER_NAMES, out.tolist()))

    def timing(self, enable=True):
        self._check(self._L.pdfmc_timing(self._h, int(bool(enable))), "timing")

    def timing_read(self):
        ms, cnt = C.c_double(), C.c_int64()
        self._check(self._L.pdfmc_timing_read(self._h, C.byref(ms), C.byref(cnt)), "timing_read")
        return ms.value, cnt.value

    def draw_gaussians(self, seed, step, stream, ids):
        torch = self.torch
        ids_d = torch.as_tensor(np.ascontiguousarray(ids, np.uint32).view(np.int32), device=self.device)
        dt = torch.float64 if self.prec == FP64 else torch.float32
        out = torch.empty((len(ids), 6), dtype=dt, device=self.device)
        self._check(self._L.pdfmc_draw_gaussians(self._h, int(seed), int(step), int(stream),
                                                 C.c_void_p(ids_d.data_ptr()), len(ids),
                                                 C.c_void_p(out.data_ptr())), "draw_gaussians")
        return out.cpu().numpy()
