"""Writes sphere1280_nearfield_interval_eigs.txt: eigenvalues kappa in [2.5, 5] of the near-field-corrected
single-layer operator (near pairs within 2 longest edges integrated over the source triangle) of
the unit icosphere at level 3 (n = 1280), by the oracle's
Chebyshev route (Algorithm 2 inside Algorithm 3 with restarts, reduced pencil
eq. sc1_chebyshev_red; N = 32 first-kind nodes, shift at the centre, q = 10,
tol = 1e-12, seed-1 starting block of 16 columns).  Calls only the oracle; run from the
repository root:
    python tests/golden/make_sphere1280_nearfield_interval_eigs.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import method as M  # noqa: E402


def main():
    xyz, tri = synth.icosphere(3)
    op = M.Operator(xyz, tri, nearfield_eta=2.0)
    V = synth.probe_block(op.n, 16, seed=1)
    lam, X, res, outer, _ = M.cheb_subspace_iteration(op, 2.5, 5.0, 32, V, q=10, tol=1e-12,
                                                      imag_tol=1e-2, verbose=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere1280_nearfield_interval_eigs.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle eigenvalues of T_nf(kappa) x = 0 (near pairs within 2 longest edges integrated over the\n")
        fh.write("# source triangle) for the unit icosphere, level 3 (n = 1280),\n")
        fh.write("# kappa in [2.5, 5] (|Im kappa| <= 1e-2 (b - a)): Chebyshev interpolant with N = 32\n")
        fh.write("# first-kind nodes, Algorithm 2 (shift xi = 0) in Algorithm 3, q = 10, tol = 1e-12,\n")
        fh.write(f"# starting block synth.probe_block(1280, 16, seed=1); {outer} outer iterations.\n")
        fh.write("# Written by tests/golden/make_sphere1280_nearfield_interval_eigs.py (oracle only).\n")
        fh.write("# columns: Re(lambda) Im(lambda) relative_residual\n")
        for l, r in zip(lam, res):
            fh.write(f"{l.real:.17e} {l.imag:.17e} {r:.3e}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
