"""Pins of the oracle's LU with partial pivoting (oracle.method.lu_partial_pivoting and
lu_solve_factors), CPU only: a hand-worked 3 x 3 case, agreement with LAPACK's zgetrf and
zgetrs (through SciPy) in pivots and factors, P A = L U, the pivot measure
|Re| + |Im| on a case where the modulus would choose differently, ties, an all-zero
column, and planted mistakes that the pins catch."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import method as M


def _rand(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def _perm_from_ipiv(ipiv):
    p = np.arange(ipiv.size)
    for j, q in enumerate(ipiv):
        p[[j, q]] = p[[q, j]]
    return p


def _reconstruction_error(A, LU, ipiv):
    n = A.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return np.linalg.norm(A[_perm_from_ipiv(ipiv)] - L @ U) / np.linalg.norm(A)


def test_hand_worked_three_by_three():
    # rows swapped (0, 2), then (1, 2); multipliers 1/7, 4/7 and 1/2; U's last entry -1/2
    A = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 10]], dtype=np.complex128)
    for scale in (1.0, 1.0 + 1.0j):
        LU, ipiv = M.lu_partial_pivoting(scale * A)
        assert list(ipiv) == [2, 2, 2]
        L_ref = np.array([[0, 0, 0], [1 / 7, 0, 0], [4 / 7, 1 / 2, 0]])
        U_ref = np.array([[7, 8, 10], [0, 6 / 7, 11 / 7], [0, 0, -1 / 2]]) * scale
        assert np.allclose(np.tril(LU, -1), L_ref, rtol=0, atol=1e-15)
        assert np.allclose(np.triu(LU), U_ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 17, 64, 129])
def test_matches_lapack(n):
    A = _rand(n, 100 + n)
    LU, ipiv = M.lu_partial_pivoting(A)
    LU_ref, piv_ref = sla.lu_factor(A)
    assert np.array_equal(ipiv, piv_ref)
    assert np.abs(LU - LU_ref).max() <= 1e-12 * max(1.0, np.abs(LU_ref).max())
    assert _reconstruction_error(A, LU, ipiv) <= 1e-14 * n
    # |l| <= |a| / |p| <= (|Re a| + |Im a|) / (|p| ) <= (|Re p| + |Im p|) / |p| <= sqrt 2
    assert np.abs(np.tril(LU, -1)).max() <= np.sqrt(2.0) * (1.0 + 1e-15)
    B = _rand(n, 7)[:, : min(n, 5)]
    X = M.lu_solve_factors(LU, ipiv, B)
    assert np.abs(X - sla.lu_solve((LU_ref, piv_ref), B)).max() <= 1e-10 * np.abs(X).max()
    assert np.linalg.norm(A @ X - B) <= 1e-12 * n * np.linalg.norm(A) * np.linalg.norm(X)
    x = M.lu_solve_factors(LU, ipiv, B[:, 0])
    assert x.shape == (n,) and np.abs(x - X[:, 0]).max() <= 1e-12 * np.abs(X).max()


def test_pivot_measure_and_ties():
    # |Re| + |Im|: 0.75 + 0.75i (1.5) beats 1.2 (1.2), although its modulus (1.06) is smaller
    A = np.array([[0.75 + 0.75j, 1.0], [1.2, 3.0]])
    _, ipiv = M.lu_partial_pivoting(A)
    assert ipiv[0] == 0 and sla.lu_factor(A)[1][0] == 0
    # equal measures (1 and i): the first row stays
    A = np.array([[1.0, 2.0], [1.0j, 5.0]])
    _, ipiv = M.lu_partial_pivoting(A)
    assert ipiv[0] == 0 and sla.lu_factor(A)[1][0] == 0


def test_zero_column():
    A = _rand(6, 3)
    A[:, 2] = 0.0
    LU, ipiv = M.lu_partial_pivoting(A)
    assert ipiv[2] == 2 and LU[2, 2] == 0.0 and np.all(LU[3:, 2] == 0.0)
    assert _reconstruction_error(A, LU, ipiv) <= 1e-14


def test_planted_mistakes_are_caught(monkeypatch):
    """Exchanging rows only to the right of the pivot column (L's rows left unswapped), or
    pivoting on the modulus, fails the pins above."""
    A = _rand(40, 5)
    orig = M.lu_partial_pivoting

    def no_l_swap(A):
        A = np.array(A, dtype=np.complex128)
        n = A.shape[0]
        ipiv = np.zeros(n, dtype=np.int64)
        for j in range(n):
            p = j + int(np.argmax(np.abs(A[j:, j].real) + np.abs(A[j:, j].imag)))
            ipiv[j] = p
            A[[j, p], j:] = A[[p, j], j:]
            A[j + 1:, j] /= A[j, j]
            A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
        return A, ipiv

    LU, ipiv = no_l_swap(A)
    assert _reconstruction_error(A, LU, ipiv) > 1e-3

    def modulus_pivot(A):
        A = np.array(A, dtype=np.complex128)
        n = A.shape[0]
        ipiv = np.zeros(n, dtype=np.int64)
        for j in range(n):
            p = j + int(np.argmax(np.abs(A[j:, j])))
            ipiv[j] = p
            A[[j, p], :] = A[[p, j], :]
            A[j + 1:, j] /= A[j, j]
            A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
        return A, ipiv

    B = np.array([[0.75 + 0.75j, 1.0], [1.2, 3.0]])
    assert not np.array_equal(modulus_pivot(B)[1], sla.lu_factor(B)[1])
    assert np.array_equal(orig(B)[1], sla.lu_factor(B)[1])
