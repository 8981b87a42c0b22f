"""Statistical band of the node statistics (test infrastructure: used by the
tests and by the benchmark's oracle leg, never by the product path).

A node statistic is a particle estimate (reading R-11), so it carries a
sampling error set by the effective number of particles at the node,
N_eff = W^2 / sum (w lambda)^2 (W = sum w lambda, the sums over the
particles of the node's elements; the last node sum holds the denominator).
A run in another precision follows the same Wiener path, so it should sit
well inside that error of the FP64 result; the band below is k standard
errors wide:

  <U_i>                var u_i / N_eff
  <u_i u_i>            2 <u_i u_i>^2 / N_eff                (Gaussian fourth moment)
  <u_i u_j>, i != j    (<u_i u_i><u_j u_j> + <u_i u_j>^2) / N_eff   (same)
  <omega>              <omega>^2 / (4 N_eff)                (spread of the Gamma(4) initial draw)
  <psi_a>              <psi_a'^2> / N_eff
  <psi_a'^2>           <psi_a'^2> / N_eff                   (bound for |psi_a'| <= 1)

plus an absolute floor of atol times the statistic's scale, for nodes where
the statistic vanishes on both sides.
"""
import numpy as np

GROUPS = ("mean_U", "reynolds_stress", "mean_omega", "mean_psi", "psi_variance")


def columns(ns):
    """Columns of the statistics readback in each group."""
    return {"mean_U": [2, 3, 4], "reynolds_stress": [5, 6, 7, 8, 9, 10], "mean_omega": [11],
            "mean_psi": list(range(12, 12 + ns)), "psi_variance": list(range(12 + ns, 12 + 2 * ns))}


def n_eff(sums, ns):
    W = sums[:, 0]
    q = sums[:, 11 + 2 * ns]
    return np.where(q > 0.0, W * W / np.maximum(q, 1e-300), 0.0)


def sigma(st, sums, ns):
    """Standard error of each statistic at each node, same shape as st."""
    ne = np.maximum(n_eff(sums, ns), 1e-300)
    s2 = np.zeros_like(st)
    R = st[:, 5:11]
    s2[:, 2:5] = np.maximum(st[:, 5:8], 0.0) / ne[:, None]
    s2[:, 5:8] = 2.0 * R[:, 0:3] ** 2 / ne[:, None]
    for c, (i, j) in {8: (0, 1), 9: (0, 2), 10: (1, 2)}.items():
        s2[:, c] = (np.abs(R[:, i] * R[:, j]) + st[:, c] ** 2) / ne
    s2[:, 11] = st[:, 11] ** 2 / (4.0 * ne)
    for a in range(ns):
        var = np.maximum(st[:, 12 + ns + a], 0.0)
        s2[:, 12 + a] = var / ne
        s2[:, 12 + ns + a] = var / ne
    return np.sqrt(s2)


def fractions(g, r, sums, ns, rows=None, k=3.0, atol=1e-6):
    """Per group, the fraction of (node, statistic) pairs where |g - r| lies
    within k standard errors of the reference r (plus the absolute floor),
    and the largest |g - r| / sigma; rows selects the statistics nodes."""
    if rows is not None:
        g, r, sums = g[rows], r[rows], sums[rows]
    sig = sigma(r, sums, ns)
    out = {}
    for name, cols in columns(ns).items():
        if not cols:
            continue
        d = np.abs(g[:, cols] - r[:, cols])
        scale = np.maximum(np.abs(r[:, cols]).max(), 1e-300)
        ok = d <= k * sig[:, cols] + atol * scale
        z = d / np.maximum(sig[:, cols], 1e-300)
        out[name] = dict(fraction=float(ok.mean()), max_sigma=float(z.max()), median_sigma=float(np.median(z)))
    return out
