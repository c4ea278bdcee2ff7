"""Pins of the oracle's discretised operator T(kappa): agreement of its two evaluation
paths, the single-layer eigen-relations of the sphere (which the discrete operator must
approach at second order in h), analytic derivatives, and uneven meshes (CPU only)."""
import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

import synth


def _sphere_eig(l, k):
    """Eigenvalue of the single-layer operator on the unit sphere for degree l:
    S_k Y_l = i k j_l(k) h_l(k) Y_l with h_l = j_l + i y_l (first kind)."""
    j = spherical_jn(l, k)
    h = j + 1j * spherical_yn(l, k)
    return 1j * k * j * h


def test_dense_and_matrix_free_agree(oracle_lib):
    C = oracle_lib._clib
    xyz, tri = synth.perturbed_icosphere(2, 0.15, seed=3)
    V = synth.probe_block(len(tri), 5, seed=9)
    for k in (4.0, 3.3 - 0.7j):
        T = C.dense(xyz, tri, k)
        Y = C.apply_rows(xyz, tri, k, V)
        assert np.linalg.norm(T @ V - Y) <= 1e-14 * np.linalg.norm(Y)
        rows = np.array([0, 17, 319, 5])
        assert np.allclose(C.apply_rows(xyz, tri, k, V, rows), Y[rows], rtol=0, atol=1e-15)
        # diagonal of the dense matrix is the self term
        assert np.allclose(np.diag(T), C.self_terms(xyz, tri, [k])[0], rtol=1e-15, atol=0)


@pytest.mark.parametrize("kappa", [4.0, 4.0 - 0.5j, 2.5 + 0.3j])
def test_sphere_eigen_relations_converge(oracle_lib, kappa):
    """T(k) 1 -> (sin k e^{ik}/k) 1 and T(k) z -> i k j_1 h_1 z as the icosphere is
    refined; the discretisation error must fall by about 4x per level (O(h^2))."""
    C = oracle_lib._clib
    lam0, lam1 = _sphere_eig(0, kappa), _sphere_eig(1, kappa)
    assert abs(lam0 - np.sin(kappa) * np.exp(1j * kappa) / kappa) < 1e-14 * abs(lam0)
    e0, e1 = [], []
    for L in (2, 3, 4):
        xyz, tri = synth.icosphere(L)
        n = len(tri)
        rows = np.arange(0, n, max(1, n // 64))
        y = C.apply_rows(xyz, tri, kappa, np.ones((n, 1)), rows)[:, 0]
        e0.append(np.abs(y - lam0).max() / abs(lam0))
        _, cen, _, _ = C.geometry(xyz, tri)
        z = cen[:, 2].astype(complex)
        y1 = C.apply_rows(xyz, tri, kappa, z[:, None], rows)[:, 0]
        e1.append(np.linalg.norm(y1 - lam1 * z[rows]) / np.linalg.norm(lam1 * z[rows]))
    for e in (e0, e1):
        assert e[-1] < 1e-2
        assert 3.0 < e[0] / e[1] < 5.5 and 3.0 < e[1] / e[2] < 5.5, e


def test_uneven_mesh_row_sums(oracle_lib):
    """On a sphere mesh with uneven triangle areas the row sums still approach
    sin k e^{ik}/k: the area weight must be that of the source triangle b."""
    C = oracle_lib._clib
    k = 3.7 + 0.2j
    lam0 = _sphere_eig(0, k)
    errs = []
    for L in (3, 4):
        xyz, tri = synth.perturbed_icosphere(L, 0.15, seed=11)
        n = len(tri)
        area, _, _, _ = C.geometry(xyz, tri)
        assert area.max() / area.min() > 5.0
        rows = np.arange(0, n, max(1, n // 64))
        y = C.apply_rows(xyz, tri, k, np.ones((n, 1)), rows)[:, 0]
        errs.append(np.abs(y - lam0).max() / abs(lam0))
    assert errs[-1] < 1e-2 and errs[0] / errs[1] > 3.0, errs


def test_kernel_derivative_is_analytic(oracle_lib):
    """d-th derivative in kappa (kernel (i r)^d g) against a Cauchy-integral derivative."""
    C = oracle_lib._clib
    xyz, tri = synth.icosphere(1)
    k0, rad, M = 4.2 + 0.1j, 0.6, 64
    th = 2 * np.pi * np.arange(M) / M
    Ts = np.stack([C.dense(xyz, tri, k0 + rad * np.exp(1j * t)) for t in th])
    scale = np.abs(Ts).max()
    for d in (1, 2):
        fac = float(np.prod(np.arange(1, d + 1)))
        ref = fac * np.tensordot(np.exp(-1j * d * th), Ts, axes=(0, 0)) / M / rad ** d
        got = C.dense(xyz, tri, k0, deriv=d)
        assert np.abs(got - ref).max() <= 1e-13 * scale * fac / rad ** d
