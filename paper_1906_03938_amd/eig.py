"""Eigenvalues inside a contour or in a real interval from device sweeps (the host steps of
the method).  ContourSolver below is the Cauchy form; IntervalSolver, further down, the
Chebyshev form.

Algorithm 3 of the paper with the restarts of Section 3.2: q steps of inverse iteration
on the linearisation of the Cauchy approximation (Algorithm 1) build a basis U; the
Rayleigh-Ritz blocks B^_j = w_j U^H T(z_j) U give the reduced pencil eq. sc1_cauchy_red,
solved by the QZ algorithm; Ritz pairs inside the contour are accepted when every relative
residual ||T(lambda) x|| / ||x|| is at most `tol`, otherwise the next outer iteration
restarts from them.

Every application of the BEM operator is a library sweep (contour_moments, cheb_moments, rr_project,
bem_assemble_apply), and the n x n matrix of the inverse iteration (the Schur complement S,
or G for the Chebyshev form) is generated densely on the device by bem_assemble_sum, and
factorised and solved with by the library's own LU kernels (bem_lu_factor, bem_lu_solve);
the rest of the host algebra is QR of n x nu blocks and QZ of the (N+1) nu pencil.

Inverse iteration without storing the N v-blocks.  With shift s = c, d_i = z_i - s,
B_i = w_i T(z_i) and the moment blocks M_p = sum_i B_i d_i^-p, one step of Algorithm 1 --
S u' = sum_i B_i v_i / d_i with the Schur complement S = M_1, then v_i' = (v_i - u')/d_i
(block elimination of (A - s M) w' = M w, whose bottom right-hand block is zero) -- keeps
every v-block of the form
    v_i = sum_p a_p d_i^-p + b / (lam - z_i)
(the last term only on restarts, which start from v_i = x/(lam - z_i)).  Substituting,
    u'   = S^-1 [ sum_p M_{p+1} a_p + (M_1 + R_lam) b / (lam - c) ],
    a'_1 = -u' + b/(lam - c),   a'_{p+1} = a_p,   b' = b/(lam - c),
with R_lam = sum_i B_i/(lam - z_i).  So a_p at step j is the a_1 created at step j-p+1,
and each new a_1 is swept once with every moment order it will still be needed for.
Columns are not normalised between steps (a per-column scale does not change the span the
Rayleigh-Ritz step uses); only the final block is orthonormalised.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import _lib

# size of the Cauchy pencil above which Rayleigh-Ritz takes the shift-invert Arnoldi route
DENSE_QZ_MAX = 1200


def _host(t):
    """Host (numpy) copy of a device tensor, through a pinned buffer of torch's caching host
    allocator: a copy into pageable memory runs at a fraction of the link's rate.  CPU
    tensors (the driver's tests) are returned as they are."""
    import torch

    if not t.is_cuda:
        return t.numpy()
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t)
    return h.numpy()


def _device(a):
    """Device copy of a host array (complex128), staged through pinned memory."""
    import torch

    h = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).pin_memory()
    return h.to("cuda", non_blocking=True)


def _combine_blocks(combine, blocks, coef):
    """sum_b coef[b][c] blocks[b][:, c] through `combine` (at most 64 blocks per call: longer
    sums continue from the previous partial sum as their first block)."""
    blocks = list(blocks)
    coef = np.asarray(coef, dtype=np.complex128)
    out = combine(blocks[:64], coef[:64])
    one = np.ones((1, coef.shape[1]), dtype=np.complex128)
    for b0 in range(64, len(blocks), 63):
        out = combine([out] + blocks[b0:b0 + 63], np.concatenate([one, coef[b0:b0 + 63]]), out=out)
    return out


class DenseFactor:
    """LU factorisation P S = L U (partial pivoting) of the dense n x n complex matrix of the
    inverse iteration, held on the device, with solves for host right-hand sides.  "device"
    (and "auto"): the library's own kernels (bem_lu_factor, bem_lu_solve), in place -- the
    matrix passed in is overwritten by its factors, so no second n x n array is needed, and
    every index is 64-bit, so n is bounded by memory only.  "host": SciPy (LAPACK) on a host
    copy, for driver tests without a GPU."""

    def __init__(self, S, mode="auto"):
        self.mode = "device" if mode == "auto" else mode
        if self.mode == "device":
            self.lu = _lib.LU(S)
            info = self.lu.info
            if info:
                raise np.linalg.LinAlgError(f"matrix is singular to working precision (pivot column {info - 1})")
        elif self.mode == "host":
            self.lu = sla.lu_factor(S.cpu().numpy())
        else:
            raise ValueError(f"unknown LU mode {mode!r}")

    def solve(self, B):
        B = np.asarray(B, dtype=np.complex128)
        if self.mode == "host":
            return sla.lu_solve(self.lu, B)
        vec = B.ndim == 1
        X = _host(self.lu.solve(_device(B.reshape(B.shape[0], -1))))
        return X[:, 0] if vec else X

    def solve_t(self, B):
        """S^-1 B for an n x m tensor B: on the device in "device" mode (the result stays
        there), through SciPy on a CPU tensor in "host" mode."""
        if self.mode == "host":
            import torch

            return torch.from_numpy(sla.lu_solve(self.lu, B.numpy()))
        return self.lu.solve(B)


def _assemble(mesh, z, c, flags):
    """sum_j c_j T(z_j) on the device, generated directly in FP64 (bem_assemble_sum) with the
    sweeps' form.  The matrix the LU factorises stays FP64 when the sweeps run at reduced
    precision: the inverse iteration's subspace is then as accurate as those sweeps, and the
    matrix costs one generation pass instead of a reduced-precision sweep of the n x n
    identity."""
    return mesh.assemble_sum(z, c, form=flags & ~_lib.PREC_MASK)


def _nearfield_add(mesh, model, z, W, Xd, out):
    """out += sum_j W[j, p] dT(z_j) Xd: the quadrature's correction (model None) or the
    network's inside the trust region of `model` (a nfnet.NearFieldNet)."""
    if model is None:
        mesh.nearfield_moments(z, W, Xd, out=out)
    else:
        mesh.nearfield_moments_net(model.c_model(), z, W, Xd, out=out)
    return out


def _residuals(mesh, dev, lam, X, chunk=16, nearfield=False, model=None):
    """Relative residuals ||T(lam_k) x_k|| / ||x_k||.  Up to `chunk` pairs share one
    bem_assemble_apply call (all their wavenumbers applied to all their vectors, the diagonal
    kept): the direct sweep generates its operators in blocks of 8, so one call per pair would
    generate 8 operators for each.  nearfield: T is the operator with the mesh's near-field
    correction (added with per-node weights: dT(lam_k) X), by the quadrature or by `model`."""
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.empty(lam.size)
    for k0 in range(0, lam.size, chunk):
        k1 = min(lam.size, k0 + chunk)
        Xd = dev(X[:, k0:k1])
        Y = mesh.assemble_apply(lam[k0:k1], Xd)
        if nearfield:
            _nearfield_add(mesh, model, lam[k0:k1], np.eye(k1 - k0), Xd, Y)
        Y = _host(Y)
        for k in range(k0, k1):
            out[k] = np.linalg.norm(Y[k - k0, :, k - k0]) / np.linalg.norm(X[:, k])
    return out


class ContourSolver:
    """Cauchy-approximation eigensolver for T(kappa) x = 0 inside |kappa - c| < radius,
    with N trapezoidal nodes, q inverse-iteration steps per outer iteration."""

    def __init__(self, mesh, c, radius, N, q=10, tol=1e-12, max_outer=30, sweep_prec=0, rr_prec=0, lu="auto",
                 nearfield=False):
        import torch

        self.torch = torch
        self.mesh = mesh
        # solve with the mesh's near-field-corrected operator: True for the quadrature's
        # correction, a trained nfnet.NearFieldNet for the network's (the quadrature outside its
        # trust region; S keeps the quadrature's correction)
        self.nf_model = nearfield if hasattr(nearfield, "c_model") else None
        self.nearfield = self.nf_model is not None or bool(nearfield)
        self.n = mesh.n
        self.c = complex(c)
        self.radius = float(radius)
        self.N = int(N)
        self.q = int(q)
        self.tol = float(tol)
        self.max_outer = int(max_outer)
        self.z, self.w, self.W = _lib.contour_nodes(self.c, self.radius, self.N, shift=self.c, P=self.q + 1)
        self.sweep_flags = int(sweep_prec)  # arithmetic of the subspace sweeps (moments, S)
        self.rr_flags = int(rr_prec)        # arithmetic of the Rayleigh-Ritz projections
        self._S_lu = None
        self.lu_mode = lu
        self.history = []

    def _dev(self, a):
        return _device(a)

    # -- sweeps -------------------------------------------------------------------
    def _moments_t(self, Xd, orders, sign=1.0):
        """M_p X (sign +1) or M_p (-X) (sign -1, the weights negated: exact) for moment orders
        p >= 1, X a device block: one contour_moments sweep; the result stays on the device."""
        W = np.ascontiguousarray(sign * self.W[:, [p - 1 for p in orders]])
        M = self.mesh.contour_moments(self.z, W, Xd, form=self.sweep_flags)
        if self.nearfield:
            _nearfield_add(self.mesh, self.nf_model, self.z, W, Xd, M)
        return M

    def moments(self, X, orders):
        """M_p X for moment orders p >= 1 (host arrays): one contour_moments sweep of X."""
        return _host(self._moments_t(self._dev(X), orders))

    def r_lam(self, x, lam):
        """Columns R_lam_k x_k = sum_i w_i T(z_i) x_k / (lam_k - z_i), k < x.shape[1]: one sweep
        of the block with one weight set per column (column k of weight set k is kept)."""
        return _host(self._moments_and_r_lam_t(self._dev(x), [], lam)[1])

    def moments_and_r_lam(self, x, orders, lam):
        """(M_p x for the moment orders, R_lam x as r_lam) from one sweep of x (host arrays)."""
        M, R = self._moments_and_r_lam_t(self._dev(x), orders, lam)
        return _host(M), _host(R)

    def _moments_and_r_lam_t(self, xd, orders, lam):
        """The moment weight sets and the per-column resolvent weight sets side by side in one
        contour_moments call (the unfolded sweep's cost does not depend on the number of
        weight sets); both results stay on the device."""
        lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
        Wm = self.W[:, [p - 1 for p in orders]]
        Wr = self.w[:, None] / (lam[None, :] - self.z[:, None])
        W = np.ascontiguousarray(np.concatenate([Wm, Wr], axis=1))
        M = self.mesh.contour_moments(self.z, W, xd, form=self.sweep_flags)
        if self.nearfield:
            _nearfield_add(self.mesh, self.nf_model, self.z, W, xd, M)
        P = len(orders)
        k = self.torch.arange(lam.size, device=M.device)
        return M[:P], M[P + k, :, k].T.contiguous()

    def _combine(self, blocks, coef, out=None):
        """sum_b coef[b][c] blocks[b][:, c] on the device (bem_block_combine; out may be the
        first block)."""
        return _lib.block_combine(blocks, coef, out=out)

    def schur_lu(self):
        """LU of S = M_1 = sum_i B_i/(z_i - c), assembled on the device."""
        if self._S_lu is None:
            S = _assemble(self.mesh, self.z, self.W[:, 0], self.sweep_flags)
            if self.nearfield:
                self.mesh.nearfield_sum(self.z, self.W[:, 0], S)
            self._S_lu = DenseFactor(S, self.lu_mode)
            del S
        return self._S_lu

    # -- Algorithm 1, q steps -------------------------------------------------------
    def inverse_iteration(self, u0, lam=None):
        """u after q steps from v_i = u0/(c - z_i) (lam None) or v_i = u0/(lam_k - z_i).  The
        swept moment blocks, the right-hand sides and the iterates stay on the device (the
        right-hand side of each step is one bem_block_combine of the swept blocks); only the
        final block comes back."""
        lu = self.schur_lu()
        q = self.q
        restart = lam is not None
        m = np.asarray(u0).shape[1]
        one = np.ones(m, dtype=np.complex128)
        swept = []  # swept[k][o] = M_{o+2} a_1^(k), device
        if restart:
            rho = 1.0 / (np.asarray(lam, dtype=np.complex128) - self.c)  # per column
            xd = self._dev(np.asarray(u0, dtype=np.complex128))
            Mx, Rx = self._moments_and_r_lam_t(xd, list(range(1, q + 2)), lam)  # M_1 x .. M_{q+1} x, R_lam x
            base = self._combine([Mx[0], Rx], np.stack([one, one]))      # (M_1 + R_lam) x
            swept.append(None)                                           # no a_1^(0) on restarts
        else:
            swept.append(self._moments_t(self._dev(u0), list(range(2, q + 2)), sign=-1.0))  # a_1^(0) = -u0
        u = None
        for j in range(q):
            blocks = [swept[k][j - k] for k in range(j + 1) if swept[k] is not None]  # M_{j-k+2} a_1^(k)
            coef = [one] * len(blocks)
            if restart:
                blocks.append(base)
                coef.append(rho ** (j + 1))
            acc = self._combine(blocks, np.stack(coef))
            u = lu.solve_t(acc)
            if j + 1 < q:
                orders = list(range(2, q - j + 1))                       # still needed by steps j+1 .. q-1
                Ma = self._moments_t(u, orders, sign=-1.0)               # a_1 = -u
                if restart:                                              # a_1 += x rho^(j+1)
                    for o in range(len(orders)):
                        self._combine([Ma[o], Mx[1 + o]], np.stack([one, rho ** (j + 1)]), out=Ma[o])
                swept.append(Ma)
        return np.asarray(u0) if u is None else _host(u)

    # -- Rayleigh-Ritz ---------------------------------------------------------------
    def reduced_pencil(self, Bhat):
        """eq. sc1_cauchy_red over all N nodes: unknowns [v^_0 .. v^_{N-1}, y]."""
        N, m = len(Bhat), Bhat[0].shape[0]
        A = np.zeros(((N + 1) * m, (N + 1) * m), dtype=np.complex128)
        M = np.zeros_like(A)
        eye = np.eye(m)
        for j in range(N):
            sl = slice(j * m, (j + 1) * m)
            A[sl, sl] = self.z[j] * eye
            A[sl, N * m:] = eye
            A[N * m:, sl] = -Bhat[j]
            M[sl, sl] = eye
        return A, M

    def ritz_shift_invert(self, Bhat, k):
        """The k eigenvalues of the reduced pencil closest to the centre c and their y-parts,
        without the dense QZ (whose cost grows as ((N+1) m)^3).  Shift-invert at c:
        (A - c M)^-1 M has the finite eigenvalues theta = 1/(lam - c), and on the v-part it is
        D^-1 - D^-1 E G^-1 B D^-1 with D = (Z - c) (x) I, E = 1 (x) I, B = [B^_0 .. B^_{N-1}]
        and G = sum_j B^_j/(z_j - c) (block elimination of the arrow-shaped pencil), so a
        product costs O(N m^2); ARPACK takes the k largest |theta|.  The y-part of the pencil
        eigenvector belonging to v is G^-1 B D^-1 v."""
        from scipy.sparse.linalg import LinearOperator, eigs

        N, m = len(Bhat), Bhat[0].shape[0]
        d = 1.0 / (self.z - self.c)
        Bh = np.stack(Bhat)
        G_lu = sla.lu_factor(np.einsum("j,jab->ab", d, Bh))

        def y_of(F):  # G^-1 B D^-1 v for block rows F (N x m x cols)
            return sla.lu_solve(G_lu, np.einsum("jab,jbc->ac", Bh, d[:, None, None] * F))

        def matvec(f):
            F = f.reshape(N, m, 1)
            DF = d[:, None, None] * F
            y = y_of(F)
            return (DF - d[:, None, None] * y[None, :, :]).reshape(-1)

        op = LinearOperator((N * m, N * m), matvec=matvec, dtype=np.complex128)
        theta, Xv = eigs(op, k=k, which="LM", ncv=min(N * m, max(2 * k + 1, 40)), tol=0.0)
        Y = y_of(Xv.reshape(N, m, k))
        return self.c + 1.0 / theta, Y

    def rayleigh_ritz(self, U):
        Ud = self._dev(U)
        P = self.mesh.rr_project(self.z, Ud, form=self.rr_flags)
        if self.nearfield:
            self.mesh.nearfield_project(self.z, Ud, P, None if self.nf_model is None else self.nf_model.c_model())
        P = _host(P)
        Bhat = [self.w[j] * P[j] for j in range(self.N)]
        m = U.shape[1]
        if (self.N + 1) * m > DENSE_QZ_MAX:
            return self.ritz_shift_invert(Bhat, min(m, self.N * m - 2))
        A, M = self.reduced_pencil(Bhat)
        with np.errstate(invalid="ignore", divide="ignore"):
            lam, V = sla.eig(A, M)
        Y = V[-m:, :]
        return lam, Y

    def residuals(self, lam, X):
        return _residuals(self.mesh, self._dev, lam, X, nearfield=self.nearfield, model=self.nf_model)

    # -- Algorithm 3 with restarts -------------------------------------------------------
    def solve(self, U0):
        u0 = np.asarray(U0, dtype=np.complex128)
        nu = u0.shape[1]
        lam_restart = None
        for outer in range(self.max_outer):
            u = self.inverse_iteration(u0, lam_restart)
            U, _ = np.linalg.qr(u)
            lam, Y = self.rayleigh_ritz(U)
            finite = np.isfinite(lam)
            inside = finite & (np.abs(lam - self.c) < self.radius)
            Yin = Y[:, inside]
            X = U @ (Yin / np.linalg.norm(Yin, axis=0, keepdims=True))
            lam_in = lam[inside]
            res = self.residuals(lam_in, X)
            self.history.append((lam_in.copy(), res.copy()))
            if lam_in.size and res.max() <= self.tol:
                order = np.argsort(lam_in.real)
                return lam_in[order], X[:, order], res[order], outer + 1
            idx = np.flatnonzero(finite)[np.argsort(np.abs(lam[finite] - self.c))][:nu]
            Yr = Y[:, idx]
            u0 = U @ (Yr / np.linalg.norm(Yr, axis=0, keepdims=True))
            lam_restart = lam[idx]
        order = np.argsort(lam_in.real)
        return lam_in[order], X[:, order], res[order], self.max_outer


def eigs_in_contour(mesh, c, radius, N, U0, q=10, tol=1e-12, max_outer=30, sweep_prec=0, rr_prec=0, lu="auto",
                    nearfield=False):
    """(eigenvalues, eigenvectors, relative residuals, outer iterations) of T(kappa) x = 0
    inside |kappa - c| < radius; U0 is the n x nu starting block.  sweep_prec / rr_prec are
    the library's precision flags (PREC_*) for the subspace sweeps and for the Rayleigh-Ritz
    projections; residuals are always evaluated in FP64.  lu: where the Schur complement is
    factorised ("host", "device" or "auto", see DenseFactor).  nearfield: solve with the
    operator corrected on the mesh's near-pair list (Mesh.set_nearfield) in every sweep, in S,
    the projections and the residuals: True for the quadrature's correction, a trained
    nfnet.NearFieldNet for the network's (quadrature outside its trust region and in S)."""
    return ContourSolver(mesh, c, radius, N, q=q, tol=tol, max_outer=max_outer, sweep_prec=sweep_prec,
                         rr_prec=rr_prec, lu=lu, nearfield=nearfield).solve(U0)


class IntervalSolver:
    """Chebyshev-interpolation eigensolver for T(kappa) x = 0 with kappa in [a, b]: the
    degree d = N-1 interpolant at first-kind nodes (eq. Chebyshev), q steps of Algorithm 2
    per outer iteration with the shift xi = `shift` (0 is the centre of the interval,
    kappa = alpha + beta xi), Rayleigh-Ritz with eq. sc1_chebyshev_red and restarts.

    Algorithm 2 without storing the d v-blocks.  Block elimination of (A - s M) w' = M w for
    the linearisation eq. sc1_chebyshev gives v'_l = T_l(s) v'_0 + p_l with p_0 = 0,
    p_1 = v_0, p_{l+1} = 2 s p_l - p_{l-1} + 2 v_l, and G v'_0 = -sum_{l=0}^{d} B_l p_l with
    G = sum_l B_l T_l(s).  Every block is a combination of earlier iterates h_k with scalar
    coefficients, v_l = sum_k g_k[l] h_k, and each coefficient vector evolves on its own:
    g' = (p_0 .. p_{d-1}) of the recurrence driven by g.  So an iterate of age a (swept a
    steps after it was made) enters the right-hand side as sum_j T(kappa_j) W_a[j] h_k with
    W_a[j] = -sum_l coef[l, j] p^(a)_l, a table fixed once s is chosen: each new iterate is
    swept once (contour_moments on the Chebyshev nodes) with all the ages it will reach.
    A restart block x_k = Ritz vector with its own xi_k has per-column coefficients
    g[l] = T_l(xi_k); it is swept once by cheb_moments (all B_l x) and combined on the host."""

    def __init__(self, mesh, a, b, N, q=10, tol=1e-12, max_outer=30, shift=0.0, imag_tol=1e-2, sweep_prec=0,
                 rr_prec=0, lu="auto", nearfield=False):
        import torch

        if N < 3:
            raise ValueError("the Chebyshev pencil needs N >= 3 nodes")
        self.torch = torch
        self.mesh = mesh
        self.nearfield = bool(nearfield)  # solve with the mesh's near-field-corrected operator
        self.n = mesh.n
        self.a, self.b, self.N = float(a), float(b), int(N)
        self.alpha, self.beta = 0.5 * (self.a + self.b), 0.5 * (self.b - self.a)
        self.q = int(q)
        self.tol = float(tol)
        self.max_outer = int(max_outer)
        self.s = complex(shift)
        self.imag_tol = float(imag_tol)
        self.d = self.N - 1
        self.sweep_flags = int(sweep_prec)
        self.rr_flags = int(rr_prec)
        kappa, self.coef = _lib.cheb_nodes(self.a, self.b, self.N)
        self.z = kappa.astype(np.complex128)
        self.t_s = self._tvals(self.s)                              # T_0(s) .. T_d(s)
        self.W_age = np.empty((self.N, self.q), dtype=np.complex128)
        g = self.t_s[:self.d].copy()
        for age in range(self.q):
            p = self._drive(g[:, None])[:, 0]
            self.W_age[:, age] = -(self.coef.T @ p)
            g = p[:self.d]
        self._G_lu = None
        self.lu_mode = lu
        self.history = []

    def _tvals(self, xi):
        """T_0(xi) .. T_d(xi) (xi scalar or per-column vector: rows l, columns k)."""
        xi = np.asarray(xi, dtype=np.complex128)
        out = np.empty((self.d + 1,) + xi.shape, dtype=np.complex128)
        out[0] = 1.0
        if self.d >= 1:
            out[1] = xi
        for l in range(2, self.d + 1):
            out[l] = 2 * xi * out[l - 1] - out[l - 2]
        return out

    def _drive(self, g):
        """p_0 .. p_d of the recurrence driven by block coefficients g (d x k)."""
        p = np.zeros((self.d + 1, g.shape[1]), dtype=np.complex128)
        p[1] = g[0]
        for l in range(1, self.d):
            p[l + 1] = 2 * self.s * p[l] - p[l - 1] + 2 * g[l]
        return p

    def _dev(self, a):
        return _device(a)

    def _sweep_t(self, Xd, ages):
        """Age sweeps of a device block (contour_moments on the Chebyshev nodes); the result
        stays on the device."""
        W = np.ascontiguousarray(self.W_age[:, list(ages)])
        M = self.mesh.contour_moments(self.z, W, Xd, form=self.sweep_flags)
        if self.nearfield:
            self.mesh.nearfield_moments(self.z, W, Xd, out=M)
        return M

    def sweep(self, X, ages):
        return _host(self._sweep_t(self._dev(X), ages))

    def _combine(self, blocks, coef, out=None):
        """sum_b coef[b][c] blocks[b][:, c] on the device (bem_block_combine; out may be the
        first block)."""
        return _lib.block_combine(blocks, coef, out=out)

    def g_lu(self):
        """LU of G = sum_l B_l T_l(s) = sum_j T(kappa_j) sum_l coef[l, j] T_l(s), assembled on
        the device."""
        if self._G_lu is None:
            wg = self.coef.T @ self.t_s
            G = _assemble(self.mesh, self.z, wg, self.sweep_flags)
            if self.nearfield:
                self.mesh.nearfield_sum(self.z, wg, G)
            self._G_lu = DenseFactor(G, self.lu_mode)
            del G
        return self._G_lu

    def inverse_iteration(self, u0, xi=None):
        """u after q steps of Algorithm 2 from v_l = T_l(s) u0 (xi None) or from the restart
        blocks v_l = T_l(xi_k) u0[:, k].  The swept blocks, right-hand sides and iterates stay
        on the device (bem_block_combine forms the right-hand sides and the restart terms);
        only the final block comes back."""
        lu = self.g_lu()
        q = self.q
        u0 = np.asarray(u0, dtype=np.complex128)
        one = np.ones(u0.shape[1], dtype=np.complex128)
        swept = []                                   # swept[k][a]: age-a sweep of iterate k (device)
        restart = None
        if xi is None:
            swept.append(self._sweep_t(self._dev(u0), range(q)))
        else:
            u0d = self._dev(u0)
            Cx = self.mesh.cheb_moments(self.a, self.b, self.N, self.N, u0d, form=self.sweep_flags)
            if self.nearfield:  # C_l += sum_k coef[l, k] dT(kappa_k) u0
                self.mesh.nearfield_moments(self.z, np.ascontiguousarray(self.coef.T), u0d, out=Cx)
            g = self._tvals(np.asarray(xi, dtype=np.complex128))[:self.d]   # d x m
            restart = []
            for _ in range(q):
                p = self._drive(g)                   # -sum_l p[l, k] C_l[:, k]
                restart.append(_combine_blocks(self._combine, [Cx[l] for l in range(self.N)], -p))
                g = p[:self.d]
            swept.append(None)
        u = None
        for j in range(q):
            blocks = [swept[k][j - k] for k in range(j + 1) if swept[k] is not None]
            if restart is not None:
                blocks.append(restart[j])
            rhs = _combine_blocks(self._combine, blocks, np.stack([one] * len(blocks)))
            u = lu.solve_t(rhs)
            if j + 1 < q:
                swept.append(self._sweep_t(u, range(q - 1 - j)))
        return u0 if u is None else _host(u)

    def reduced_pencil(self, Bhat):
        """eq. sc1_chebyshev_red: unknowns [y, v_1 .. v_{d-1}]; rows xi y = v_1,
        2 xi v_l = v_{l-1} + v_{l+1}, and 2 xi B_d v_{d-1} = B_d v_{d-2} - sum_{l<d} B_l v_l."""
        d, m = self.d, Bhat.shape[1]
        A = np.zeros((d * m, d * m), dtype=np.complex128)
        M = np.zeros_like(A)
        eye = np.eye(m)
        A[:m, m:2 * m] = eye
        M[:m, :m] = eye
        for l in range(1, d - 1):
            r = slice(l * m, (l + 1) * m)
            A[r, (l - 1) * m:l * m] = eye
            A[r, (l + 1) * m:(l + 2) * m] = eye
            M[r, r] = 2 * eye
        last = slice((d - 1) * m, d * m)
        for l in range(d):
            A[last, l * m:(l + 1) * m] = -Bhat[l]
        A[last, (d - 2) * m:(d - 1) * m] += Bhat[d]
        M[last, last] = 2 * Bhat[d]
        return A, M

    def rayleigh_ritz(self, U):
        """kappa and y of the reduced pencil with B_hat_l = sum_j coef[l, j] U^H T(kappa_j) U."""
        Ud = self._dev(U)
        P = self.mesh.rr_project(self.z, Ud, form=self.rr_flags)
        if self.nearfield:
            self.mesh.nearfield_project(self.z, Ud, P)
        P = _host(P)
        Bhat = np.einsum("lj,jab->lab", self.coef, P)
        A, M = self.reduced_pencil(Bhat)
        with np.errstate(invalid="ignore", divide="ignore"):
            xi, V = sla.eig(A, M)
            kap = self.alpha + self.beta * xi
        return kap, V[:U.shape[1], :]

    def residuals(self, lam, X):
        return _residuals(self.mesh, self._dev, lam, X, nearfield=self.nearfield)

    def solve(self, U0):
        u0 = np.asarray(U0, dtype=np.complex128)
        nu = u0.shape[1]
        xi = None
        centre = self.alpha + self.beta * self.s
        for outer in range(self.max_outer):
            u = self.inverse_iteration(u0, xi)
            U, _ = np.linalg.qr(u)
            lam, Y = self.rayleigh_ritz(U)
            finite = np.isfinite(lam)
            with np.errstate(invalid="ignore"):
                inside = (finite & (lam.real >= self.a) & (lam.real <= self.b)
                          & (np.abs(lam.imag) <= self.imag_tol * (self.b - self.a)))
            Yin = Y[:, inside]
            X = U @ (Yin / np.linalg.norm(Yin, axis=0, keepdims=True))
            lam_in = lam[inside]
            res = self.residuals(lam_in, X)
            self.history.append((lam_in.copy(), res.copy()))
            if lam_in.size and res.max() <= self.tol:
                order = np.argsort(lam_in.real)
                return lam_in[order], X[:, order], res[order], outer + 1
            idx = np.flatnonzero(finite)[np.argsort(np.abs(lam[finite] - centre))][:nu]
            Yr = Y[:, idx]
            u0 = U @ (Yr / np.linalg.norm(Yr, axis=0, keepdims=True))
            xi = (lam[idx] - self.alpha) / self.beta
        order = np.argsort(lam_in.real)
        return lam_in[order], X[:, order], res[order], self.max_outer


def eigs_in_interval(mesh, a, b, N, U0, q=10, tol=1e-12, max_outer=30, shift=0.0, imag_tol=1e-2, sweep_prec=0,
                     rr_prec=0, lu="auto", nearfield=False):
    """(eigenvalues, eigenvectors, relative residuals, outer iterations) of T(kappa) x = 0
    with kappa in [a, b] (|Im kappa| <= imag_tol (b - a)), from the Chebyshev interpolant
    with N first-kind nodes; U0 is the n x nu starting block.  sweep_prec / rr_prec / lu /
    nearfield as for eigs_in_contour."""
    return IntervalSolver(mesh, a, b, N, q=q, tol=tol, max_outer=max_outer, shift=shift,
                          imag_tol=imag_tol, sweep_prec=sweep_prec, rr_prec=rr_prec, lu=lu,
                          nearfield=nearfield).solve(U0)
