"""GPU tests of the library's dense LU with partial pivoting (bem_lu_factor, bem_lu_solve)
against the oracle's unblocked elimination (oracle.method.lu_partial_pivoting, pinned to
LAPACK in test_oracle_lu.py), through the C ABI.

* Parity at sizes that span several 32-column sub-panels and 256-column panels with ragged
  tails: pivots and the permutation bit-exact, factors within 1e-12 of max |U| (the same
  pivots, different rounding orders), P A = L U normwise to n x 1e-16, solves within 1e-10
  relative of the oracle's solve with its own factors.
* Edge cases: n = 1, a row stride larger than n, strided right-hand sides, an all-zero
  column (info = its index + 1, factors still equal to the oracle's), an exact tie, bitwise
  reproducibility, argument errors.
* n = 12288 (one panel boundary at 12288 = 48 x 256; 2.4 GB), at the tiles the eigen-solver
  uses: ||A x - b|| / (||A|| ||x||) below 1e-14 for 64 right-hand sides, and the pivots of
  the first 64 columns equal the oracle's on the same matrix (computed column-wise below)."""
import ctypes

import numpy as np
import pytest

from oracle import method as M

pytestmark = pytest.mark.gpu


def _rand(n, seed, cols=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, n if cols is None else cols)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _perm(ipiv):
    p = np.arange(ipiv.size)
    for j, q in enumerate(ipiv):
        p[[j, q]] = p[[q, j]]
    return p


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1906_03938_amd as bem
    from paper_1906_03938_amd import _lib

    assert torch.cuda.is_available()
    return torch, bem, _lib


def _factor(env, A, pad=0):
    torch, bem, _lib = env
    n = A.shape[0]
    buf = torch.zeros((n, n + pad), dtype=torch.complex128, device="cuda")
    buf[:, :n] = torch.from_numpy(A).to("cuda")
    lu = _lib.LU(buf[:, :n])
    return lu, buf


@pytest.mark.parametrize("n", [1, 31, 33, 255, 257, 600])
def test_factor_and_solve_match_oracle(env, n):
    torch, bem, _lib = env
    A = _rand(n, 1000 + n)
    print(f"LU parity n = {n}", flush=True)
    lu, buf = _factor(env, A, pad=3 if n > 1 else 0)
    info = lu.info
    LU = buf[:, :n].cpu().numpy()
    ipiv = lu.ipiv.cpu().numpy()
    perm = lu.perm.cpu().numpy()
    LU_ref, ipiv_ref = M.lu_partial_pivoting(A)
    assert info == 0
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.array_equal(perm, _perm(ipiv_ref))
    scale = np.abs(LU_ref).max()
    assert np.abs(LU - LU_ref).max() <= 1e-12 * scale, np.abs(LU - LU_ref).max() / scale
    L = np.tril(LU, -1) + np.eye(n)
    assert np.linalg.norm(A[perm] - L @ np.triu(LU)) <= n * 1e-16 * np.linalg.norm(A) + 1e-300
    # strided right-hand sides (ldb = m + 2) and output (ldx = m + 1)
    m = 7
    B = _rand(n, 5, cols=m)
    Bd = torch.zeros((n, m + 2), dtype=torch.complex128, device="cuda")
    Bd[:, :m] = torch.from_numpy(B).to("cuda")
    Xd = torch.zeros((n, m + 1), dtype=torch.complex128, device="cuda")
    lu.solve(Bd[:, :m], out=Xd[:, :m])
    X = Xd[:, :m].cpu().numpy()
    X_ref = M.lu_solve_factors(LU_ref, ipiv_ref, B)
    assert np.abs(X - X_ref).max() <= 1e-10 * np.abs(X_ref).max()
    assert np.all(Xd[:, m].cpu().numpy() == 0) and np.all(Bd[:, m:].cpu().numpy() == 0)


def test_zero_column_and_tie(env):
    torch, bem, _lib = env
    n = 70
    A = _rand(n, 77)
    A[:, 40] = 0.0
    # column 0: rows 3 and 9 tie in |Re| + |Im| and beat every other row
    A[:, 0] *= 0.1
    A[3, 0], A[9, 0] = 4.0 + 1.0j, -2.0 + 3.0j
    lu, buf = _factor(env, A)
    LU = buf.cpu().numpy()
    ipiv = lu.ipiv.cpu().numpy()
    LU_ref, ipiv_ref = M.lu_partial_pivoting(A)
    assert ipiv_ref[0] == 3 and ipiv_ref[40] == 40
    assert lu.info == 41
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.abs(LU - LU_ref).max() <= 1e-12 * np.abs(LU_ref).max()


def test_reproducible_and_errors(env):
    torch, bem, _lib = env
    n = 300
    A = _rand(n, 3)
    lu1, b1 = _factor(env, A)
    lu2, b2 = _factor(env, A)
    assert torch.equal(b1, b2) and torch.equal(lu1.ipiv, lu2.ipiv)
    B = torch.from_numpy(_rand(n, 4, cols=5)).to("cuda")
    assert torch.equal(lu1.solve(B), lu2.solve(B))
    L = _lib.lib()
    w = torch.empty(L.bem_lu_work_bytes(n, 0), dtype=torch.uint8, device="cuda")
    p = [ctypes.c_void_p(t.data_ptr()) for t in (lu1.ipiv, lu1.perm, lu1._info)]
    before = b1.clone()
    # lda < n, host work, work too small: refused before anything is launched
    assert L.bem_lu_factor(ctypes.c_void_p(b1.data_ptr()), n, n - 1, *p, ctypes.c_void_p(w.data_ptr()), w.numel(),
                           None) == _lib.BEM_EINVAL
    hostw = np.zeros(w.numel(), dtype=np.uint8)
    assert L.bem_lu_factor(ctypes.c_void_p(b1.data_ptr()), n, n, *p, hostw.ctypes.data_as(ctypes.c_void_p),
                           w.numel(), None) == _lib.BEM_EINVAL
    assert L.bem_lu_factor(ctypes.c_void_p(b1.data_ptr()), n, n, *p, ctypes.c_void_p(w.data_ptr()), 8,
                           None) == _lib.BEM_EINVAL
    assert L.bem_lu_work_bytes(0, 0) == -1 and L.bem_lu_work_bytes(5, -1) == -1
    torch.cuda.synchronize()
    assert torch.equal(b1, before)
    # X overlapping B
    with pytest.raises(bem.BemError, match="overlaps"):
        lu1.solve(B, out=B)


def test_large_n_residual(env):
    torch, bem, _lib = env
    n, m = 12288, 64
    print(f"LU n = {n}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(21)
    A = torch.complex(torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g))
    # the oracle's pivots of the first columns, from a host copy of the leading column block
    # (elimination of columns j < 64 touches only those columns and the pivot rows)
    A64 = A[:, :64].cpu().numpy()
    B = torch.complex(torch.randn((n, m), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((n, m), dtype=torch.float64, device="cuda", generator=g))
    normA = torch.linalg.matrix_norm(A).item()
    Acopy = A.clone()
    lu = _lib.LU(A)
    assert lu.info == 0
    X = lu.solve(B)
    R = Acopy @ X - B
    rel = (torch.linalg.matrix_norm(R) / (normA * torch.linalg.matrix_norm(X))).item()
    print(f"n = {n}: ||A X - B|| / (||A|| ||X||) = {rel:.2e}", flush=True)
    assert rel <= 1e-14
    _, ipiv64 = M.lu_partial_pivoting(A64)
    assert np.array_equal(lu.ipiv[:64].cpu().numpy(), ipiv64)
