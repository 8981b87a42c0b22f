"""pdfmc_sort_noalloc, the sort that allocates nothing (its temporaries live
in a static device array), against pdfmc_sort through the C ABI.

Index work, so the bar is bit-exactness: after each sort the two contexts
hold the same particles in the same order. Three calls in a row, each on a
smaller context than the last (fewer elements and particle slots), so each
call finds the previous call's contents in the shared array; the second
has segments longer than one wavefront sorts. A context too large for the
array is refused with PDFMC_E_INVALID.
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


def _context(P, mesh, params, parts, steps):
    sim = P.Sim("fp64", "cuda:0")
    cs = sim.add_case(mesh, params, len(parts["x"]))
    sim.bind()
    sim.set_options(sort_interval=0, use_graph=False)
    sim.upload(cs, parts)
    sim.init()
    sim.step(steps)
    return sim, cs


def _same(a, b):
    return all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in a)


CASES = [
    ("square-16-ppe60", 16, 60, 7),
    ("square-4-ppe700", 4, 700, 5),     # segments of ~700 particles
    ("square-3-ppe40", 3, 40, 3),
]


def test_noalloc_sort_matches_sort(P):
    last = None
    for name, nodes, ppe, steps in CASES:
        mesh = W.unit_square(nodes, 0.2, periodic_x=True, seed_key=(7, nodes, 0))
        params = W.default_params(mode=1, n_scalars=1, dt=1e-3, nu=1e-3)
        parts = W.init_particles(mesh, ppe, 1, W.rng_for(7, nodes, 1), u_std=0.1,
                                 psi_disks=[(0.5, 0.5, 0.3, 1.0)])
        n = len(parts["x"])
        if last is not None:
            assert mesh.n_elems < last[0] and n < last[1], (mesh.n_elems, n, last)
        last = (mesh.n_elems, n)
        _flush(f"[sort_noalloc] {name}: {mesh.n_elems} triangles, {n} particles, {steps} steps, then a sort")
        a, ca = _context(P, mesh, params, parts, steps)
        b, cb = _context(P, mesh, params, parts, steps)
        assert _same(a.download(ca, n), b.download(cb, n))
        a.sort()
        b.sort_noalloc()
        b.synchronize()
        ga, gb = a.download(ca, n), b.download(cb, n)
        key = gb["elem"].astype(np.int64) * (1 << 32) + gb["id"].astype(np.int64)
        assert np.all(np.diff(key) > 0)
        assert _same(ga, gb), name
        # the sorted states step alike
        a.step(2)
        b.step(2)
        assert _same(a.download(ca, n), b.download(cb, n)), name
        assert np.array_equal(a.stats(ca), b.stats(cb)), name


def test_noalloc_sort_refuses_a_context_beyond_the_array(P):
    mesh = W.unit_square(6, 0.2, periodic_x=True, seed_key=(7, 0, 0))
    sim = P.Sim("fp64", "cuda:0")
    sim.add_case(mesh, W.default_params(mode=1, n_scalars=0), 2_000_000)
    _flush("[sort_noalloc] context with 2e6 particle slots: refused")
    sim.bind()
    with pytest.raises(P.PdfmcError, match="INVALID.*static scratch"):
        sim.sort_noalloc()
