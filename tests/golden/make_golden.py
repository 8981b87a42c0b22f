"""Writes the oracle's regression record of the small square case.

The record holds the node statistics of the oracle after a few steps of a
small FP64 case (mode 1, one scalar, two cells of velocity bins), written
with 17 significant digits. It is produced by the oracle alone (nothing of
the GPU library is imported) and is a guard against unintended changes of the
oracle's arithmetic: a deliberate change regenerates it with

    python tests/golden/make_golden.py

and the commit names the passage of the paper (or the reading of it) that
justifies the change.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "small_square_oracle_stats.txt")
STEPS = 6


def case():
    import workloads as W
    mesh = W.unit_square(6, 0.2, periodic_x=True, periodic_y=False, seed_key=(80, 0, 0))
    params = W.default_params(mode=1, dt=2e-3, nu=1e-3, n_scalars=1, src=[(0.3, 0.6, 0.15, 1.0)])
    parts = W.init_particles(mesh, 12, 1, W.rng_for(80, 0, 1), u_std=0.3, psi_disks=[(0.5, 0.5, 0.2, 1.0)])
    return mesh, params, parts


def run():
    import oracle
    mesh, params, parts = case()
    o = oracle.Oracle()
    cs = o.add_case(mesh, params)
    o.upload(cs, parts)
    o.init()
    o.step(STEPS)
    return o.stats(cs)


if __name__ == "__main__":
    st = run()
    with open(OUT, "w") as f:
        f.write("# oracle node statistics of the small square case after %d steps (tests/golden/make_golden.py)\n"
                % STEPS)
        f.write("# columns: W, rho, <U1..3>, <u1u1>, <u2u2>, <u3u3>, <u1u2>, <u1u3>, <u2u3>, <omega>, <psi>, <psi'^2>\n")
        for row in st:
            f.write(" ".join("%.17g" % v for v in row) + "\n")
    print("wrote", OUT)
