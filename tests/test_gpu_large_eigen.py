"""Eigen-extraction at the full sweep size (opt-in: set BEMRAT_LARGE_TESTS=1; about 4 minutes
on one MI355X, of which 23 s is the LU): sphere-81920 (unit icosphere level 6), the circle
|z - 5| = 2 with N = 64 trapezoidal nodes, 32 probes (seed 2), q = 10, tol 1e-12.  The Schur
complement S (107 GB) is generated on the device and factorised in place by the library's
LU (bem_lu_factor); every inverse-iteration step solves with it (bem_lu_solve).

Properties checked (the oracle cannot run at this size): 17 eigenvalues, every relative
residual ||T(lambda) x|| / ||x|| at most 1e-12, the multiplicities of the unit sphere's
interior Dirichlet eigenvalues j_l(kappa) = 0 in (3, 7) -- 1 (l = 0), 3 (l = 1), 5 (l = 2),
1 (l = 0, second zero), and the l = 3 septet split 3 + 4 by the icosahedral mesh -- each
cluster within 1e-8 (relative) and within 5e-4 of the continuum value (the discretisation
error at level 6)."""
import os

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("BEMRAT_LARGE_TESTS") != "1",
                                 reason="about 4 minutes: set BEMRAT_LARGE_TESTS=1")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_sphere81920_contour_eigenvalues():
    import time

    import torch

    import paper_1906_03938_amd as bem
    from paper_1906_03938_amd.eig import ContourSolver

    assert torch.cuda.is_available()
    xyz, tri = synth.icosphere(6)
    n = tri.shape[0]
    tab = np.loadtxt(os.path.join(GOLDEN, "sphere_dirichlet_eigs.txt"))
    t0 = time.perf_counter()
    spent = {"inverse_iteration": 0.0, "rayleigh_ritz": 0.0, "residuals": 0.0}

    class Progress(ContourSolver):
        """Prints a line per outer iteration (each takes about 8 s here) and adds up the time
        of the three phases of an outer iteration."""

        def _timed(self, name, f, *a):
            t = time.perf_counter()
            out = f(*a)
            torch.cuda.synchronize()
            spent[name] += time.perf_counter() - t
            return out

        def inverse_iteration(self, u0, lam=None):
            return self._timed("inverse_iteration", super().inverse_iteration, u0, lam)

        def rayleigh_ritz(self, U):
            return self._timed("rayleigh_ritz", super().rayleigh_ritz, U)

        def residuals(self, lam, X):
            res = self._timed("residuals", super().residuals, lam, X)
            print(f"outer iteration {len(self.history) + 1}: {lam.size} Ritz values inside, max residual "
                  f"{res.max() if res.size else float('nan'):.2e}, {time.perf_counter() - t0:.0f} s", flush=True)
            return res

    with bem.Mesh(xyz, tri) as mesh:
        solver = Progress(mesh, 5.0, 2.0, 64, q=10, tol=1e-12, max_outer=40, lu="device")
        solver.schur_lu()
        torch.cuda.synchronize()
        t_lu = time.perf_counter() - t0
        print(f"n = {n}: S assembled and factorised in {t_lu:.1f} s", flush=True)
        lam, X, res, outer = solver.solve(synth.probe_block(n, 32, seed=2))
    print(f"n = {n}: {lam.size} eigenvalues after {outer} outer iterations, {time.perf_counter() - t0:.0f} s; "
          f"max residual {res.max():.2e}\n{np.sort_complex(lam)}", flush=True)
    print("time per phase: " + ", ".join(f"{k} {v:.1f} s" for k, v in spent.items()), flush=True)
    assert lam.size == 17 and res.max() <= 1e-12
    lam = np.sort_complex(lam)
    # clusters of the sorted real parts
    cuts = np.flatnonzero(np.diff(lam.real) > 1e-6 * np.abs(lam[1:]))
    sizes = np.diff(np.concatenate([[0], cuts + 1, [lam.size]]))
    assert list(sizes) == [1, 3, 5, 1, 3, 4], sizes
    groups = np.split(lam, cuts + 1)
    for g in groups:
        assert np.ptp(g.real) <= 1e-8 * abs(g[0])
    cont = [tab[np.argmin(np.abs(tab[:, 0] - g[0].real)), 0] for g in groups]
    assert np.allclose(cont[4], cont[5])  # the split septet has one continuum value
    for g, c in zip(groups, cont):
        assert abs(g[0].real - c) < 5e-4, (g[0], c)
