"""Writes box752_interval_eigs.txt: eigenvalues kappa in [6.5, 8] of the discretised
single-layer operator on the surface of the 1.0 x 0.8 x 0.6 box meshed with 10 x 8 x 6
face-grid intervals (n = 752), by the oracle's Chebyshev route (Algorithm 2 in Algorithm 3
with restarts; N = 24 first-kind nodes, shift at the centre, q = 10, tol = 1e-12,
starting block synth.probe_block(752, 8, seed=3)).  The continuum value is
pi sqrt(1 + 1/0.8^2 + 1/0.6^2) = 7.2599; the coarse mesh shifts it by about 0.006.
Calls only the oracle; run from the repository root:
    python tests/golden/make_box752_eigs.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import method as M  # noqa: E402


def main():
    xyz, tri = synth.box_surface(counts=(10, 8, 6))
    op = M.Operator(xyz, tri)
    V = synth.probe_block(op.n, 8, seed=3)
    lam, X, res, outer, _ = M.cheb_subspace_iteration(op, 6.5, 8.0, 24, V, q=10, tol=1e-12, imag_tol=1e-2)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "box752_interval_eigs.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle eigenvalues of T(kappa) x = 0 on the 1.0 x 0.8 x 0.6 box surface, 10 x 8 x 6 grid\n")
        fh.write("# (n = 752), kappa in [6.5, 8]: Chebyshev interpolant with N = 24 first-kind nodes,\n")
        fh.write(f"# Algorithm 2 in Algorithm 3, q = 10, tol = 1e-12, probe_block(752, 8, seed=3); {outer} outer.\n")
        fh.write("# Written by tests/golden/make_box752_eigs.py (oracle only).\n")
        fh.write("# columns: Re(lambda) Im(lambda) relative_residual\n")
        for l, r in zip(lam, res):
            fh.write(f"{l.real:.17e} {l.imag:.17e} {r:.3e}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
