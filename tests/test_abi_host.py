"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/pdfmc.h declares, validates meshes and arguments
before any device work, and derives the same statistics-node map (periodic
images merged) as the oracle."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_1006_0549_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1006_0549_amd import build
        build.build()
    return P


def test_exports_every_declared_symbol(pkg):
    hdr = open(os.path.join(ROOT, "include", "pdfmc.h")).read()
    declared = set(re.findall(r"\b(pdfmc_[a-z_0-9]+)\s*\(", hdr))
    assert "pdfmc_step" in declared and len(declared) >= 20
    L = pkg.lib()
    missing = [f for f in sorted(declared) if not hasattr(L, f)]
    assert not missing, missing
    assert declared == set(pkg.EXPORTS)


def _sim(pkg):
    return pkg.Sim("fp64", host_only=True)


def test_mesh_rejections(pkg):
    mesh = W.unit_square(6, 0.0, periodic_x=True)
    s = _sim(pkg)
    bad = W.Mesh("cw", mesh.xy, mesh.tri[:, [0, 2, 1]].copy(), mesh.edge_tag, mesh.bcs)
    with pytest.raises(pkg.PdfmcError, match="MESH.*counter-clockwise"):
        s.add_case(bad, W.default_params(), 10)
    bcs = [dict(b) for b in mesh.bcs]
    bcs[2] = dict(type=W.BC_PERIODIC, shift=(0.5, 0.0))
    with pytest.raises(pkg.PdfmcError, match="MESH.*partner"):
        s.add_case(W.Mesh("p", mesh.xy, mesh.tri, mesh.edge_tag, bcs), W.default_params(), 10)
    tag = mesh.edge_tag.copy()
    e, k = next((e, k) for e in range(mesh.n_elems) for k in range(3) if tag[e, k] < 0)
    tag[e, k] = 0
    with pytest.raises(pkg.PdfmcError, match="MESH"):
        s.add_case(W.Mesh("t", mesh.xy, mesh.tri, tag, mesh.bcs), W.default_params(), 10)
    tri = mesh.tri.copy()
    tri[0, 0] = mesh.n_nodes + 3
    with pytest.raises(pkg.PdfmcError, match="MESH.*references node"):
        s.add_case(W.Mesh("r", mesh.xy, tri, mesh.edge_tag, mesh.bcs), W.default_params(), 10)


def test_argument_rejections(pkg):
    mesh = W.unit_square(6, 0.0, periodic_x=True)
    s = _sim(pkg)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*n_bins"):
        s.add_case(mesh, W.default_params(n_bins=3), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*n_scalars"):
        s.add_case(mesh, W.default_params(n_scalars=5), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*dt"):
        s.add_case(mesh, W.default_params(dt=0.0), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*capacity"):
        s.add_case(mesh, W.default_params(), -1)
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.init()
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.step(1)
    with pytest.raises(pkg.PdfmcError, match="INVALID"):
        s.set_options(0, 100, False)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*block size"):
        s.set_options(0, 192, False)          # would let a workgroup span two cases
    with pytest.raises(pkg.PdfmcError, match="INVALID.*n_eff_min"):
        s.add_case(mesh, W.default_params(n_eff_min=-1.0), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*reaction"):
        s.add_case(mesh, W.default_params(reaction=3), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*reaction 2"):
        s.add_case(mesh, W.default_params(reaction=2, n_scalars=2), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*k_react"):
        s.add_case(mesh, W.default_params(reaction=1, k_react=(1.0, -2.0, 0.0, 0.0)), 10)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*tail_rows"):
        s.set_solver(0, -5)
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.autotune(2)


@pytest.mark.parametrize("which", ["square", "channel"])
def test_stat_node_map_matches_oracle(pkg, oracle_mod, which):
    mesh = W.unit_square(12, 0.2, periodic_x=True) if which == "square" else W.channel(n_half=10, nx=30)
    s = _sim(pkg)
    cs = s.add_case(mesh, W.default_params(), 100)
    nsn, sn = s.case_info(cs)
    o = oracle_mod.Oracle()
    oc = o.add_case(mesh, W.default_params())
    info = o.mesh_info(oc)
    assert nsn == info["n_stat_nodes"]
    np.testing.assert_array_equal(sn, info["stat_node"])


def test_workspace_grows_with_capacity(pkg):
    mesh = W.unit_square(8, 0.2)
    a = _sim(pkg)
    a.add_case(mesh, W.default_params(), 1000)
    b = _sim(pkg)
    b.add_case(mesh, W.default_params(), 100000)
    assert b.workspace_bytes() > a.workspace_bytes() + 2 * 99000 * 8 * 7


def test_projection_factor_host(pkg):
    """add_case factors the projection matrix of a mode-2 case on the host:
    the direct projection is the default, with a supernode tree of several
    levels and O(n log n) stored values; the method can be switched, and
    other methods are rejected."""
    cfg = W.config_channel(ppe=1, n_half=16, nx=40)
    s = _sim(pkg)
    info0 = s.projection_info()
    assert info0["factor_values"] == 0 and info0["height"] == -1
    s.add_case(cfg["mesh"], dict(cfg["params"], mode=2), 10)
    info = s.projection_info()
    assert info["method"] == "direct"
    assert info["height"] >= 3
    nsn, _ = s.case_info(0)
    assert nsn < info["factor_values"] < 200 * nsn
    s.set_projection_solver("pcg")
    assert s.projection_info()["method"] == "pcg"
    s.set_projection_solver("direct")
    with pytest.raises(ValueError):
        s.set_projection_solver("lu")
    with pytest.raises(pkg.PdfmcError, match="INVALID.*method"):
        s._check(s._L.pdfmc_set_projection_solver(s._h, 7), "set_projection_solver")


def test_upload_rejections_before_device_work(pkg):
    """The particle upload checks the whole ensemble on the host: an element
    outside the case, a bin beyond the case's bins, a non-finite value or a
    mass weight that is not positive is PDFMC_E_INVALID; a valid ensemble
    passes the checks and then meets the missing workspace (PDFMC_E_STATE)."""
    mesh = W.unit_square(6, 0.2, periodic_x=True)
    s = _sim(pkg)
    cs = s.add_case(mesh, W.default_params(n_scalars=1), 1000)
    good = W.init_particles(mesh, 3, 1, W.rng_for(0, 0, 1))
    n = len(good["x"])

    def bad(**kw):
        p = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in good.items()}
        for k, (i, v) in kw.items():
            if k == "psi":
                p[k][0, i] = v
            else:
                p[k][i] = v
        return p

    cases = [(dict(elem=(5, mesh.n_elems)), "element"), (dict(elem=(0, -1)), "element"),
             (dict(x=(7, np.nan)), "non-finite x"), (dict(omega=(n - 1, np.inf)), "non-finite omega"),
             (dict(weight=(3, 0.0)), "mass weight"), (dict(weight=(4, -1e-3)), "mass weight"),
             (dict(psi=(2, np.nan)), "non-finite scalar")]
    for kw, msg in cases:
        with pytest.raises(pkg.PdfmcError, match="INVALID.*" + msg):
            s.upload(cs, bad(**kw))
    with pytest.raises(pkg.PdfmcError, match="INVALID.*bin"):
        s.upload(cs, dict(good, bin=np.full(n, 8, np.uint8)))      # bins are 0..7
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.upload(cs, good)


def test_init_fields_and_stage_rejections(pkg):
    """Argument checks of the device initial draw, the fields upload (freeze
    bits, finiteness) and the step's stage mask."""
    mesh = W.unit_square(6, 0.2, periodic_x=True)
    s = _sim(pkg)
    cs = s.add_case(mesh, W.default_params(n_scalars=1), 10 * mesh.n_elems)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*ppe"):
        s.init_particles(cs, 0)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*capacity"):
        s.init_particles(cs, 11)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*u_std"):
        s.init_particles(cs, 2, u_std=-1.0)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*omega_scale"):
        s.init_particles(cs, 2, omega_scale=0.0)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*disk"):
        s.init_particles(cs, 2, disks=[(0.5, 0.5, np.nan, 1.0)])
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.init_particles(cs, 10)
    F = np.zeros((mesh.n_nodes, pkg.NF))
    with pytest.raises(pkg.PdfmcError, match="INVALID.*freeze_mask"):
        s.fields_upload(cs, F, freeze_mask=1 << pkg.NF)
    F[3, 7] = np.nan
    with pytest.raises(pkg.PdfmcError, match="INVALID.*non-finite"):
        s.fields_upload(cs, F)
    F[3, 7] = 0.0
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.fields_upload(cs, F, freeze_mask=(1 << pkg.NF) - 1)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*stage"):
        s.step(1, stages=8)
    with pytest.raises(pkg.PdfmcError, match="INVALID.*n_steps"):
        s.step(-1)
    with pytest.raises(pkg.PdfmcError, match="STATE"):
        s.step(1, stages=s.STAGE_ADVANCE)


def test_size_limits_rejected_on_the_host(pkg):
    """Both size limits of the scatter's sort keys are checked on the host,
    before any array beyond the sizes is read or any device memory is used:
    a case of 2^23 elements (the wavefront sort packs the element above nine
    bits of bin and lane into 32 bits) at add_case, and more than 2^29
    particle slots in one context (record keys, workgroup * 512 + position,
    stay below 2^32) at workspace_bind, which returns before it touches the
    workspace address (a placeholder here)."""
    import ctypes as C
    import types
    s = _sim(pkg)
    mesh = W.unit_square(6, 0.0, periodic_x=True)
    huge = types.SimpleNamespace(xy=mesh.xy, tri=mesh.tri, edge_tag=mesh.edge_tag, bcs=mesh.bcs,
                                 n_nodes=mesh.n_nodes, n_elems=1 << 23)
    with pytest.raises(pkg.PdfmcError, match=r"INVALID.*2\^23"):
        s.add_case(huge, W.default_params(), 10)
    s.add_case(mesh, W.default_params(), (1 << 29) + 1)
    with pytest.raises(pkg.PdfmcError, match=r"INVALID.*2\^29"):
        s._check(s._L.pdfmc_workspace_bind(s._h, C.c_void_p(256), C.c_uint64(1 << 62)), "workspace_bind")
    t = _sim(pkg)
    t.add_case(mesh, W.default_params(), 1 << 29)
    with pytest.raises(pkg.PdfmcError, match="NOMEM"):
        t._check(t._L.pdfmc_workspace_bind(t._h, C.c_void_p(256), C.c_uint64(1 << 20)), "workspace_bind")
