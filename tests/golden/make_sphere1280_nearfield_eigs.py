"""Writes sphere1280_nearfield_eigs.txt: eigenvalues of the near-field-corrected single-layer
operator (near pairs |x_a - x_b| < 2 h_b integrated over the source triangle) of the unit
icosphere at level 3 (n = 1280) inside |z - 4| < 1.5, by the oracle's Algorithm 3 (N = 32
trapezoidal nodes, q = 10, tol = 1e-12, seed-1 starting block of 16 columns).
Calls only the oracle; run from the repository root:
    python tests/golden/make_sphere1280_nearfield_eigs.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import method as M  # noqa: E402


def main():
    xyz, tri = synth.icosphere(3)
    op = M.Operator(xyz, tri, nearfield_eta=2.0)
    V = synth.probe_block(op.n, 16, seed=1)
    lam, X, res, outer, _ = M.subspace_iteration(op, 4.0, 1.5, 32, V, q=10, tol=1e-12)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere1280_nearfield_eigs.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle eigenvalues of T_nf(kappa) x = 0 (near pairs within 2 longest edges integrated\n")
        fh.write("# over the source triangle) for the unit icosphere, level 3 (n = 1280), inside\n")
        fh.write("# |kappa - 4| < 1.5: Algorithm 3, N = 32 trapezoidal nodes, q = 10, tol = 1e-12,\n")
        fh.write(f"# starting block synth.probe_block(1280, 16, seed=1); {outer} outer iterations.\n")
        fh.write("# Written by tests/golden/make_sphere1280_nearfield_eigs.py (oracle only).\n")
        fh.write("# columns: Re(lambda) Im(lambda) relative_residual\n")
        for l, r in zip(lam, res):
            fh.write(f"{l.real:.17e} {l.imag:.17e} {r:.3e}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
