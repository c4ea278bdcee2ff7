"""Plain FP64 reference for the contour / Chebyshev approximation method of El-Guide,
Miedlar and Saad, "A rational approximation method for solving acoustic nonlinear
eigenvalue problems" (arXiv 1906.03938).

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU-baseline leg
may import this module.  It never imports the product package.

Every function below writes out the plain definition it cites.  Dense linear algebra
(matrix products, LU, QR, the QZ algorithm) is delegated to NumPy/SciPy as library
primitives inside the method's steps; the LU with partial pivoting is also written out
(lu_partial_pivoting) as the reference of the library's own factorisation.  The BEM
operator comes from the C core in bem_oracle.c.

Readings of passages that are ambiguous or garbled in the paper (each one is listed in
the design notes):
  * circle nodes are trapezoidal with a half-step offset, theta_j = 2 pi (j + 1/2) / N;
  * the weight of the Cauchy rule written as sum_j w_j T(s_j)/(z - s_j) is
    w_j = -(s_j - c)/N on a circle and w_j = i s'(theta_j)/N on an ellipse;
  * the Schur complement and the right-hand side of one inverse-power step are derived
    by block elimination of (A - s M) w' = M w; the bottom block of M w is zero, so the
    right-hand side has no u term;
  * the first inverse-power iterate uses v_i = u/(s - sigma_i), the restart uses
    v_i = x/(lambda - sigma_i);
  * Chebyshev interpolation uses first-kind nodes and DCT-II coefficients.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import _clib

# ----------------------------------------------------------------------------------
# Nodes and weights (Section 2, eq. Tz, eq. TzApp, eq. Chebyshev)
# ----------------------------------------------------------------------------------


def circle_nodes(c: complex, radius: float, N: int):
    """Trapezoidal rule for the Cauchy integral eq. Tz on the circle |t - c| = radius:
    t = c + R e^{i theta}, dt = i (t - c) d theta, step 2 pi / N, so that
    T(z) ~ sum_j w_j T(s_j) / (z - s_j) (eq. TzApp) with w_j = -(s_j - c)/N."""
    theta = 2.0 * np.pi * (np.arange(N) + 0.5) / N
    s = c + radius * np.exp(1j * theta)
    w = -(s - c) / N
    return s, w


def ellipse_nodes(c: complex, rx: float, ry: float, N: int):
    """Trapezoidal rule on the ellipse s(theta) = c + rx cos(theta) + i ry sin(theta):
    (1/2 pi i) sum_j T(s_j) s'(theta_j) (2 pi / N) / (s_j - z) gives w_j = i s'(theta_j)/N
    in the form of eq. TzApp."""
    theta = 2.0 * np.pi * (np.arange(N) + 0.5) / N
    s = c + rx * np.cos(theta) + 1j * ry * np.sin(theta)
    ds = -rx * np.sin(theta) + 1j * ry * np.cos(theta)
    return s, 1j * ds / N


def moment_weights(s, w, shift: complex, P: int):
    """W[j, p-1] = w_j (s_j - shift)^{-p}, p = 1..P: the weights that turn the node sweep
    sum_j W[j,p] T(s_j) into the blocks sum_i B_i (s_i - shift)^{-p} used by the
    inverse-power step (Algorithm 1 with B_i = w_i T(s_i))."""
    d = np.asarray(s) - shift
    p = np.arange(1, P + 1)
    return np.asarray(w)[:, None] * d[:, None] ** (-p[None, :])


def cheb_nodes(a: float, b: float, N: int):
    """First-kind Chebyshev points on [a, b] and the DCT-II coefficient matrix of the
    degree N-1 interpolant (eq. Chebyshev): kappa_k = alpha + beta cos(pi (k+1/2)/N),
    coef[l, k] = (eps_l / N) cos(pi l (k + 1/2) / N), eps_0 = 1, eps_l = 2."""
    alpha, beta = 0.5 * (a + b), 0.5 * (b - a)
    k = np.arange(N)
    kappa = alpha + beta * np.cos(np.pi * (k + 0.5) / N)
    l = np.arange(N)
    eps = np.where(l == 0, 1.0, 2.0)
    coef = (eps[:, None] / N) * np.cos(np.pi * l[:, None] * (k[None, :] + 0.5) / N)
    return kappa, coef


def cheb_eval(coefs, xi):
    """sum_l coefs[l] T_l(xi) by the three-term recurrence (coefs may be matrices)."""
    xi = complex(xi)
    t_prev, t_cur = 1.0, xi
    out = coefs[0] * t_prev
    if len(coefs) > 1:
        out = out + coefs[1] * t_cur
    for l in range(2, len(coefs)):
        t_prev, t_cur = t_cur, 2.0 * xi * t_cur - t_prev
        out = out + coefs[l] * t_cur
    return out


# ----------------------------------------------------------------------------------
# The operator and the sweep outputs (the definitions the GPU sweep must reproduce)
# ----------------------------------------------------------------------------------


class Operator:
    """T(kappa) of a closed triangle mesh; caches dense matrices for small meshes.

    nearfield_eta > 0 selects the near-field-corrected operator: the entries of the near
    pairs (|x_a - x_b| < eta h_b) are the adaptive integrals over the source triangle instead
    of their 7-point values (dense matrices only, no derivatives)."""

    def __init__(self, xyz, tri, nearfield_eta: float = 0.0):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.n = self.tri.shape[0]
        self.nearfield_eta = float(nearfield_eta)
        self._dense = {}

    def dense(self, kappa, deriv: int = 0):
        key = (complex(kappa), deriv)
        T = self._dense.get(key)
        if T is None:
            T = _clib.dense(self.xyz, self.tri, kappa, deriv)
            if self.nearfield_eta > 0.0:
                if deriv:
                    raise NotImplementedError("no derivatives of the near-field-corrected operator")
                rp, col, dT = _clib.nearfield_correction(self.xyz, self.tri, self.nearfield_eta, [kappa])
                rows = np.repeat(np.arange(self.n), np.diff(rp))
                T[rows, col] += dT[0]
            if self.n <= 2048:
                self._dense[key] = T
        return T

    def apply(self, kappa, V, rows=None, deriv: int = 0):
        """Y = T(kappa) V (rows `rows` only if given).  Small meshes use the dense matrix
        and a library matrix product; large meshes use the compensated matrix-free loop."""
        V = np.asarray(V, dtype=np.complex128)
        if rows is None and self.n <= 2048:
            return self.dense(kappa, deriv) @ V
        if self.nearfield_eta > 0.0:
            raise NotImplementedError("the near-field-corrected operator is dense only")
        return _clib.apply_rows(self.xyz, self.tri, kappa, V, rows, deriv)


def assemble_apply(op: Operator, kappas, V, rows=None):
    """Y[k] = T(kappa_k) V for each wavenumber (the plain node evaluation)."""
    return np.stack([op.apply(k, V, rows) for k in np.atleast_1d(kappas)])


def contour_moments(op: Operator, s, W, V, rows=None):
    """M_p = sum_j W[j,p] T(s_j) V (eq. TzApp with B_j = w_j T(s_j), folded with the
    per-node weights of the inverse-power step)."""
    W = np.asarray(W, dtype=np.complex128)
    Y = assemble_apply(op, s, V, rows)
    return np.einsum("jp,jam->pam", W, Y)


def cheb_moments(op: Operator, a: float, b: float, N: int, L: int, V, rows=None):
    """C_l = sum_k coef[l,k] T(kappa_k) V, l < L: the coefficient blocks B_l V of the
    Chebyshev interpolant eq. Chebyshev applied to V."""
    kappa, coef = cheb_nodes(a, b, N)
    Y = assemble_apply(op, kappa, V, rows)
    return np.einsum("lk,kam->lam", coef[:L], Y)


def rr_project(op: Operator, s, U):
    """P_j = U^H T(s_j) U (Section 3, B_hat_j = w_j P_j)."""
    U = np.asarray(U, dtype=np.complex128)
    return np.stack([U.conj().T @ op.apply(z, U) for z in np.atleast_1d(s)])


# ----------------------------------------------------------------------------------
# Linearisations and the projected eigenproblem (Section 2 and Section 3.1)
# ----------------------------------------------------------------------------------


def cauchy_pencil(Bs, s):
    """Linearisation eq. sc1_cauchy / eq. sc1_cauchy_red of sum_j B_j/(z - s_j):
    unknowns [v_0; ...; v_{N-1}; u], A = [[diag(s_j I), 1 (x) I], [-B_0 ... -B_{N-1}, 0]],
    M = diag(I, ..., I, 0)."""
    N = len(Bs)
    m = Bs[0].shape[0]
    A = np.zeros(((N + 1) * m, (N + 1) * m), dtype=np.complex128)
    M = np.zeros_like(A)
    I = np.eye(m)
    for j in range(N):
        A[j * m:(j + 1) * m, j * m:(j + 1) * m] = s[j] * I
        A[j * m:(j + 1) * m, N * m:] = I
        A[N * m:, j * m:(j + 1) * m] = -Bs[j]
        M[j * m:(j + 1) * m, j * m:(j + 1) * m] = I
    return A, M


def cheb_pencil(Bs):
    """Linearisation eq. sc1_chebyshev_red of sum_{l=0}^{d} B_l T_l(xi), d = len(Bs)-1 >= 2,
    from T_1 = xi T_0 and T_{l+1} = 2 xi T_l - T_{l-1}: unknowns [y, v_1, ..., v_{d-1}],
    rows xi v_0 = v_1, 2 xi v_l = v_{l-1} + v_{l+1}, and
    2 xi B_d v_{d-1} = -sum_{l<d} B_l v_l + B_d v_{d-2}."""
    d = len(Bs) - 1
    if d < 2:
        raise ValueError("Chebyshev pencil needs degree >= 2")
    m = Bs[0].shape[0]
    I = np.eye(m)
    A = np.zeros((d * m, d * m), dtype=np.complex128)
    M = np.zeros_like(A)
    A[0:m, m:2 * m] = I
    M[0:m, 0:m] = I
    for l in range(1, d - 1):
        A[l * m:(l + 1) * m, (l - 1) * m:l * m] = I
        A[l * m:(l + 1) * m, (l + 1) * m:(l + 2) * m] = I
        M[l * m:(l + 1) * m, l * m:(l + 1) * m] = 2 * I
    r = (d - 1) * m
    for l in range(d):
        A[r:, l * m:(l + 1) * m] = -Bs[l]
    A[r:, (d - 2) * m:(d - 1) * m] += Bs[d]
    M[r:, (d - 1) * m:] = 2 * Bs[d]
    return A, M


def solve_cauchy_reduced(Bhat, s, c, radius):
    """Eigenvalues of the reduced Cauchy pencil inside |z - c| < radius and the projected
    eigenvectors y (last block of w), by the QZ algorithm (scipy.linalg.eig)."""
    A, M = cauchy_pencil(Bhat, s)
    lam, W = sla.eig(A, M)
    m = Bhat[0].shape[0]
    ok = np.isfinite(lam) & (np.abs(lam - c) < radius)
    Y = W[-m:, ok]
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    return lam[ok], Y, lam, W[-m:, :]


def solve_cheb_reduced(Bhat, a, b, imag_tol=1e-8):
    """Eigenvalues kappa = alpha + beta xi of the reduced Chebyshev pencil with kappa in
    [a, b] and |Im kappa| <= imag_tol (b - a); y is the first block of w.  Returns
    (kappa inside, y inside, every kappa, every y)."""
    A, M = cheb_pencil(Bhat)
    with np.errstate(invalid="ignore", divide="ignore"):
        xi, W = sla.eig(A, M)
    m = Bhat[0].shape[0]
    alpha, beta = 0.5 * (a + b), 0.5 * (b - a)
    with np.errstate(invalid="ignore"):
        kap = alpha + beta * xi
    ok = (np.isfinite(kap) & (kap.real >= a) & (kap.real <= b)
          & (np.abs(kap.imag) <= imag_tol * (b - a)))
    Y = W[:m, ok]
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    return kap[ok], Y, kap, W[:m, :]


def relative_residual(op: Operator, lam, x):
    """||T(lambda) x||_2 / ||x||_2 (Section 4, accuracy measure)."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1, 1)
    return float(np.linalg.norm(op.apply(lam, x)) / np.linalg.norm(x))


# ----------------------------------------------------------------------------------
# Subspace construction: Algorithm 1 (corrected) inside Algorithm 3 with restarts
# ----------------------------------------------------------------------------------


def lu_partial_pivoting(A):
    """Gaussian elimination with row pivoting, P A = L U, of the one matrix inverse iteration
    factorises before its q steps (the Schur complement S of eq. sc3-sc4, or G of the
    Chebyshev form; Section 3).  Column by column: the pivot is the row i >= j with the
    largest |Re a_ij| + |Im a_ij| (the first of equal ones), rows j and the pivot row are
    exchanged across the whole matrix, then every row i > j gets l_ij = a_ij / a_jj and loses
    l_ij times row j.  Returns (LU, ipiv) in LAPACK's layout: L's multipliers below the
    diagonal, U on and above it, ipiv[j] the row exchanged with row j at step j (0-based).
    An all-zero candidate column leaves row j in place and its multipliers zero.  A
    rectangular A takes min(rows, columns) steps (the pivots of the leading columns do not
    depend on the columns after them)."""
    A = np.array(A, dtype=np.complex128)
    n = min(A.shape)
    ipiv = np.zeros(n, dtype=np.int64)
    for j in range(n):
        col = np.abs(A[j:, j].real) + np.abs(A[j:, j].imag)
        p = j + int(np.argmax(col))
        ipiv[j] = p
        if p != j:
            A[[j, p], :] = A[[p, j], :]
        if A[j, j] != 0:
            A[j + 1:, j] = A[j + 1:, j] / A[j, j]
        else:
            A[j + 1:, j] = 0.0
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
    return A, ipiv


def lu_solve_factors(LU, ipiv, B):
    """A^-1 B from the factors of lu_partial_pivoting: the row exchanges applied to B in
    order, forward substitution with the unit lower L, backward substitution with U."""
    X = np.array(B, dtype=np.complex128)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n = LU.shape[0]
    for j in range(n):
        p = int(ipiv[j])
        if p != j:
            X[[j, p], :] = X[[p, j], :]
    for i in range(n):
        X[i] -= LU[i, :i] @ X[:i]
    for i in range(n - 1, -1, -1):
        X[i] = (X[i] - LU[i, i + 1:] @ X[i + 1:]) / LU[i, i]
    return X[:, 0] if vec else X


def inverse_power_step(Bs, s, shift, v, u, S_lu=None):
    """One step of Algorithm 1: solve (A - shift M) w' = M w with w = [v_0..v_{N-1}; u].
    Block elimination with D = diag((s_i - shift) I), F = [I; ...; I], B = [-B_0 ... ],
    C = 0 gives the Schur complement S = sum_i B_i/(s_i - shift) (eq. linsyssim) and,
    since the bottom block of M w vanishes, the right-hand side
    b = sum_i B_i v_i/(s_i - shift) (eq. wjp1); then v_i' = (v_i - u')/(s_i - shift)
    (eq. viupd).  Returns (v', u')."""
    d = np.asarray(s) - shift
    if S_lu is None:
        S_lu = sla.lu_factor(sum(Bs[i] / d[i] for i in range(len(Bs))))
    b = sum(Bs[i] @ v[i] / d[i] for i in range(len(Bs)))
    u_new = sla.lu_solve(S_lu, b)
    v_new = [(v[i] - u_new) / d[i] for i in range(len(Bs))]
    return v_new, u_new


def subspace_iteration(op: Operator, c, radius, N, U0, q=10, tol=1e-12, max_outer=30,
                       verbose=False):
    """Algorithm 3 with the outer restarts of Section 3.2, for the Cauchy approximation on
    the circle |z - c| = radius with N trapezoidal nodes and shift = c (Section 4).

    Each outer iteration runs q steps of Algorithm 1 on every column of W (the v-blocks
    start as u/(c - s_i) on the first pass and as x/(lambda - s_i) on restarts), keeps
    the u parts, orthonormalises them (QR), projects B_hat_i = U^H B_i U, solves the
    reduced pencil eq. sc1_cauchy_red and stops once every eigenpair found inside the
    contour has relative residual ||T(lambda) x|| / ||x|| <= tol."""
    s, w = circle_nodes(c, radius, N)
    Bs = [w[j] * op.dense(s[j]) for j in range(N)]
    d = s - c
    S_lu = sla.lu_factor(sum(Bs[i] / d[i] for i in range(N)))
    u = np.array(U0, dtype=np.complex128)
    nu = u.shape[1]
    v = [u / (c - s[i]) for i in range(N)]
    history = []
    for outer in range(max_outer):
        for _ in range(q):
            v, u = inverse_power_step(Bs, s, c, v, u, S_lu)
            scale = 1.0 / np.linalg.norm(u, axis=0)
            u = u * scale
            v = [vi * scale for vi in v]
        Q, _ = np.linalg.qr(u)
        Bhat = [Q.conj().T @ B @ Q for B in Bs]
        lam_in, Y_in, lam_all, Y_all = solve_cauchy_reduced(Bhat, s, c, radius)
        X = Q @ Y_in
        res = np.array([relative_residual(op, lam_in[k], X[:, k]) for k in range(lam_in.size)])
        history.append((lam_in.copy(), res.copy()))
        if verbose:
            print(f"outer {outer}: {lam_in.size} eigenvalues, max residual "
                  f"{res.max() if res.size else float('nan'):.2e}", flush=True)
        if lam_in.size and res.max() <= tol:
            order = np.argsort(lam_in.real)
            return lam_in[order], X[:, order], res[order], outer + 1, history
        # restart from the nu finite Ritz pairs closest to the centre
        fin = np.isfinite(lam_all)
        idx = np.flatnonzero(fin)[np.argsort(np.abs(lam_all[fin] - c))][:nu]
        Xr = Q @ (Y_all[:, idx] / np.linalg.norm(Y_all[:, idx], axis=0, keepdims=True))
        lr = lam_all[idx]
        u = Xr
        v = [Xr / (lr[None, :] - s[i]) for i in range(N)]
    order = np.argsort(lam_in.real)
    return lam_in[order], X[:, order], res[order], max_outer, history


def cheb_inverse_power_step(Bs, shift, v, G_lu=None):
    """One step of Algorithm 2 (inverse power step for the Chebyshev linearisation
    eq. sc1_chebyshev) with shift s in the xi variable: solve (A - s M) w' = M w for
    w = [v_0 (= u); v_1; ...; v_{d-1}], d = len(Bs) - 1, by block elimination.

    The first d-1 block rows are the three-term recurrence of the T_l, so
    v'_l = T_l(s) v'_0 + p_l with p_0 = 0, p_1 = v_0, p_{l+1} = 2 s p_l - p_{l-1} + 2 v_l.
    Extending the recurrence to p_d, the last block row becomes
    T~(s) v'_0 = -sum_{l=0}^{d} B_l p_l with T~(s) = sum_l B_l T_l(s) (at s = 0 this is the
    matrix G of eq. Gmtx up to sign, and the right-hand side that eq. bodd / eq. beven
    write out for the two parities of d).  Returns v'."""
    d = len(Bs) - 1
    s = complex(shift)
    t = [1.0 + 0j, s]
    for _ in range(2, d + 1):
        t.append(2 * s * t[-1] - t[-2])
    if G_lu is None:
        G_lu = sla.lu_factor(sum(Bs[l] * t[l] for l in range(d + 1)))
    p = [np.zeros_like(v[0]), v[0]]
    for l in range(1, d):
        p.append(2 * s * p[l] - p[l - 1] + 2 * v[l])
    rhs = -sum(Bs[l] @ p[l] for l in range(1, d + 1))
    u_new = sla.lu_solve(G_lu, rhs)
    return [t[l] * u_new + p[l] for l in range(d)]


def cheb_subspace_iteration(op: Operator, a, b, N, U0, q=10, tol=1e-12, max_outer=30,
                            shift=0.0, imag_tol=1e-3, verbose=False):
    """Algorithm 3 for the Chebyshev interpolant of degree d = N-1 on [a, b] (Section 3):
    q steps of Algorithm 2 per outer iteration with shift xi = `shift` (0 is the centre of
    the interval, kappa = alpha + beta xi), QR of the u parts, B_hat_l = U^H B_l U, the
    reduced pencil eq. sc1_chebyshev_red, and restarts from the Ritz pairs nearest the
    centre until every accepted pair has relative residual <= tol.

    The iteration starts from v_l = T_l(s) u (the block structure of an eigenvector of the
    linearisation at xi = s) and restarts from v_l = T_l(xi_k) x_k.  Ritz values are
    accepted in [a, b] with |Im kappa| <= imag_tol (b - a)."""
    kappa, coef = cheb_nodes(a, b, N)
    alpha, beta = 0.5 * (a + b), 0.5 * (b - a)
    Ts = [op.dense(k) for k in kappa]
    Bs = [sum(coef[l, k] * Ts[k] for k in range(N)) for l in range(N)]
    del Ts
    d = N - 1
    s = complex(shift)
    G_lu = sla.lu_factor(cheb_eval(Bs, s))
    u = np.array(U0, dtype=np.complex128)
    nu = u.shape[1]

    def structured(x, xi):
        xi = np.broadcast_to(np.asarray(xi, dtype=np.complex128), (x.shape[1],))
        blocks, tp, tc = [x], np.ones_like(xi), xi
        for l in range(1, d):
            blocks.append(x * tc[None, :])
            tp, tc = tc, 2 * xi * tc - tp
        return blocks

    v = structured(u, s)
    history = []
    for outer in range(max_outer):
        for _ in range(q):
            v = cheb_inverse_power_step(Bs, s, v, G_lu)
            scale = 1.0 / np.linalg.norm(v[0], axis=0)
            v = [vl * scale for vl in v]
        Q, _ = np.linalg.qr(v[0])
        Bhat = [Q.conj().T @ B @ Q for B in Bs]
        lam_in, Y_in, lam_all, Y_all = solve_cheb_reduced(Bhat, a, b, imag_tol)
        X = Q @ Y_in
        res = np.array([relative_residual(op, lam_in[k], X[:, k]) for k in range(lam_in.size)])
        history.append((lam_in.copy(), res.copy()))
        if verbose:
            print(f"outer {outer}: {lam_in.size} eigenvalues, max residual "
                  f"{res.max() if res.size else float('nan'):.2e}", flush=True)
        if lam_in.size and res.max() <= tol:
            order = np.argsort(lam_in.real)
            return lam_in[order], X[:, order], res[order], outer + 1, history
        fin = np.isfinite(lam_all)
        idx = np.flatnonzero(fin)[np.argsort(np.abs(lam_all[fin] - (alpha + beta * s)))][:nu]
        Xr = Q @ (Y_all[:, idx] / np.linalg.norm(Y_all[:, idx], axis=0, keepdims=True))
        v = structured(Xr, (lam_all[idx] - alpha) / beta)
    order = np.argsort(lam_in.real)
    return lam_in[order], X[:, order], res[order], max_outer, history


# ----------------------------------------------------------------------------------
# Brute-force references for small meshes
# ----------------------------------------------------------------------------------


def mslp(op: Operator, kappa0, iters=30, tol=1e-14):
    """Method of successive linear problems (Ruhe): solve T(k) x = mu T'(k) x, take the
    smallest |mu| and update k <- k - mu; T' is the analytic derivative in kappa."""
    k = complex(kappa0)
    for _ in range(iters):
        mu = sla.eigvals(op.dense(k), op.dense(k, deriv=1))
        mu = mu[np.isfinite(mu)]
        step = mu[np.argmin(np.abs(mu))]
        k = k - step
        if abs(step) <= tol * abs(k):
            break
    return k


def argument_count(op: Operator, c, radius, nodes=256):
    """(1/2 pi i) contour integral of tr(T(z)^{-1} T'(z)) dz over |z - c| = radius (the
    argument principle for det T), by the trapezoidal rule."""
    s, w = circle_nodes(c, radius, nodes)
    total = 0.0j
    for j in range(nodes):
        T = _clib.dense(op.xyz, op.tri, s[j])
        dT = _clib.dense(op.xyz, op.tri, s[j], 1)
        tr = np.trace(np.linalg.solve(T, dT))
        # (1/2 pi i) f(t) dt with dt = i (t - c) 2 pi / N  ->  f(t) (t - c)/N = -w_j f(t)
        total += -w[j] * tr
    return total
