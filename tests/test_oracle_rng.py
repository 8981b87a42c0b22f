"""Pins of the oracle's Wiener-increment generator (readings R-09, R-10).

The paper only asks for Gaussian increments with zero mean and variance dt,
the same dW_i driving Eq.(2) and Eq.(4) (Sec. II). These tests tie the
oracle's counter-based generator to things other than itself:
  - its Philox4x32-10 block function to rocRAND's independent implementation
    (header source compiled here for the host),
  - its ln and sincos(2 pi .) to the C library / extended precision (<= 2 ulp),
  - the uniform and Gaussian outputs to their distributions.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ulp_diff(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.spacing(np.maximum(np.abs(a), np.abs(b)))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND pin")
    out = tmp_path_factory.mktemp("pin") / "philox_pin"
    src = os.path.join(ROOT, "tests", "pins", "philox_rocrand.cpp")
    subprocess.run([hipcc, "-O1", "-o", str(out), src], check=True, capture_output=True)
    return str(out)


def test_philox_matches_rocrand(oracle_mod, rocrand_pin):
    rng = np.random.default_rng(7)
    # the engine takes counter words 0,1 through a 64-bit offset of 4 x the
    # block index, so word 1 stays below 2^30 here (it is the step index)
    rows = rng.integers(0, 2**32, size=(400, 6), dtype=np.uint64)
    rows[:, 1] %= 2**30
    rows[:4] = [[0, 0, 0, 0, 0, 0], [1, 2, 3, 4, 5, 6],
                [2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1],
                [123456, 7, 0, 2, 10060549, 0]]
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_pin], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(t) for t in line.split()] for line in res.stdout.strip().splitlines()])
    ours = np.array([oracle_mod.philox([int(v) for v in r[:4]], [int(v) for v in r[4:]]) for r in rows])
    assert ref.shape == ours.shape
    np.testing.assert_array_equal(ours, ref)


def test_uniform_conversion_exact_and_open_interval(oracle_mod):
    # u = (2K+1) 2^-53 with K = (H << 20) | (L >> 12): reproduce K from the
    # raw Philox words and check the conversion is exact and inside (0, 1)
    seed = 10060549
    for pid, step in [(0, 0), (5, 17), (2**32 - 1, 2**31)]:
        words = []
        for blk in range(3):
            words += oracle_mod.philox([pid, step, 0, blk], [seed & 0xFFFFFFFF, seed >> 32])
        u = oracle_mod.uniform6(seed, pid, step, 0)
        for m in range(6):
            K = (words[m] << 20) | (words[6 + m] >> 12)
            assert u[m] == (2 * K + 1) * 2.0**-53
            assert 0.0 < u[m] < 1.0


def test_ln_against_libm(oracle_mod):
    rng = np.random.default_rng(1)
    us = np.concatenate([rng.random(20000), np.exp(-rng.uniform(0, 36, 20000)),
                         [2.0**-53, 0.5, 1 - 2.0**-53, 0.7071067811865476, 0.7071067811865475,
                          1.0, 2.0, 1e-300, 3.0]])
    ours = np.array([oracle_mod.ln(u) for u in us])
    ref = np.log(us.astype(np.longdouble)).astype(np.float64)
    d = _ulp_diff(ours, ref)
    d[ref == 0.0] = 0.0 if oracle_mod.ln(1.0) == 0.0 else 1e9
    assert d.max() <= 2.0, (us[np.argmax(d)], d.max())


def test_sincos2pi_against_extended_precision(oracle_mod):
    rng = np.random.default_rng(2)
    us = np.concatenate([rng.random(20000), [2.0**-53, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875,
                                             1 - 2.0**-53, 0.1, 0.3]])
    two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
    ang = two_pi * us.astype(np.longdouble)
    rs = np.sin(ang).astype(np.float64)
    rc = np.cos(ang).astype(np.float64)
    s = np.empty_like(us)
    c = np.empty_like(us)
    for i, u in enumerate(us):
        s[i], c[i] = oracle_mod.sincos2pi(u)
    # 2 ulp of the result; near a zero of sin or cos the argument x = f pi/2
    # carries one rounding, so the floor is 2 ulp of 1/2 in absolute terms
    tol_s = np.maximum(2 * np.spacing(np.abs(rs)), 2 * 2.0**-53)
    tol_c = np.maximum(2 * np.spacing(np.abs(rc)), 2 * 2.0**-53)
    assert np.all(np.abs(s - rs) <= tol_s), np.max(np.abs(s - rs) / tol_s)
    assert np.all(np.abs(c - rc) <= tol_c), np.max(np.abs(c - rc) / tol_c)
    # identity and exact quadrant points
    assert np.max(np.abs(s * s + c * c - 1.0)) < 4e-16
    assert oracle_mod.sincos2pi(0.25) == (1.0, pytest.approx(0.0, abs=1e-300))
    assert oracle_mod.sincos2pi(0.5)[1] == -1.0


def test_gaussian_moments_and_ks(oracle_mod):
    from scipy import stats
    n = 20000
    xs = np.array([oracle_mod.gauss6(10060549, i, 3, 1) for i in range(n)])
    assert xs.shape == (n, 6)
    for j in range(6):
        col = xs[:, j]
        assert abs(col.mean()) < 4 / math.sqrt(n)
        assert abs(col.var() - 1.0) < 4 * math.sqrt(2.0 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-4
    c = np.corrcoef(xs.T)
    assert np.max(np.abs(c - np.eye(6))) < 4.5 / math.sqrt(n)


def test_streams_differ_by_step_id_and_stream(oracle_mod):
    a = oracle_mod.gauss6(1, 0, 0, 0)
    assert not np.array_equal(a, oracle_mod.gauss6(1, 0, 1, 0))
    assert not np.array_equal(a, oracle_mod.gauss6(1, 1, 0, 0))
    assert not np.array_equal(a, oracle_mod.gauss6(1, 0, 0, 1))
    assert not np.array_equal(a, oracle_mod.gauss6(2, 0, 0, 0))
    np.testing.assert_array_equal(a, oracle_mod.gauss6(1, 0, 0, 0))
