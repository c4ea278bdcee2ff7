"""Pins of the oracle's method layer: the Cauchy and Chebyshev rules against closed forms,
the linearisations against known spectra, one inverse-power step against the dense
shift-and-invert operator, and the end-to-end eigenvalues against brute force and the
paper's Table 2 (CPU only)."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import jv, spherical_jn
from scipy.optimize import brentq

import synth
from oracle import method as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _poly_matrix(rng, deg, n=3):
    return [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(deg + 1)]


def _peval(A, z, deriv=0):
    out = np.zeros_like(A[0])
    for k in range(deriv, len(A)):
        out = out + A[k] * (math.factorial(k) / math.factorial(k - deriv)) * z ** (k - deriv)
    return out


def test_circle_nodes_and_weights():
    c, R, N = 4.0 + 0.5j, 1.5, 32
    s, w = M.circle_nodes(c, R, N)
    assert np.allclose(np.abs(s - c), R, rtol=1e-15)
    # sum_j w_j/(z - s_j) is the rule applied to T = 1: equals 1/(1 + zeta^N) inside
    z = c + 0.3 - 0.2j
    zeta = (z - c) / R
    assert abs(np.sum(w / (z - s)) - 1.0 / (1.0 + zeta ** N)) < 1e-14
    # outside the contour the Cauchy integral of a polynomial vanishes (up to zeta^-N)
    zo = c + 3.0 * R
    assert abs(np.sum(w / (zo - s))) < 1e-14


def test_ellipse_nodes_and_weights():
    """The trapezoidal rule on an ellipse s(theta) = c + rx cos(theta) + i ry sin(theta):
    with rx = ry it is the circle rule (same nodes and weights); the rule applied to
    T = p(z) (a polynomial) gives p(z) at points inside and 0 outside, up to the trapezoidal
    rule's geometric convergence on the periodic analytic integrand; and its first moment
    about an interior point c is -p(c), its second -p'(c) (Cauchy's formula)."""
    c, R, N = 4.0 - 0.5j, 1.5, 24
    s, w = M.ellipse_nodes(c, R, R, N)
    s0, w0 = M.circle_nodes(c, R, N)
    assert np.abs(s - s0).max() <= 1e-15 * abs(c) and np.abs(w - w0).max() <= 1e-16 * R
    rng = np.random.Generator(np.random.PCG64(11))
    coef = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    p = np.polynomial.Polynomial(coef)
    dp = p.deriv()
    c, rx, ry, N = 0.5 + 0.25j, 2.0, 1.0, 160
    s, w = M.ellipse_nodes(c, rx, ry, N)
    assert np.allclose(((s - c).real / rx) ** 2 + ((s - c).imag / ry) ** 2, 1.0, rtol=1e-15)
    for z in (c, c + 0.6 - 0.3j, c - 1.1 + 0.2j):
        approx = np.sum(w * p(s) / (z - s))
        assert abs(approx - p(z)) <= 1e-12 * abs(p(z)), z
    for z in (c + 3.0, c - 2.5j):
        assert abs(np.sum(w * p(s) / (z - s))) <= 1e-12 * np.abs(p(s)).max(), z
    W = M.moment_weights(s, w, c, 2)
    assert abs(np.sum(W[:, 0] * p(s)) + p(c)) <= 1e-12 * abs(p(c))
    assert abs(np.sum(W[:, 1] * p(s)) + dp(c)) <= 1e-12 * abs(dp(c))


def test_cauchy_rule_is_exact_on_polynomials():
    """For T of degree d < N: sum_j w_j T(s_j)/(z - s_j) = T(z)/(1 + zeta^N) with
    zeta = (z - c)/R and nodes offset by half a step."""
    rng = np.random.Generator(np.random.PCG64(1))
    c, R, N = 2.0 - 1.0j, 0.8, 16
    s, w = M.circle_nodes(c, R, N)
    A = _poly_matrix(rng, N - 1)
    for z in (c, c + 0.3 + 0.1j, c - 0.5j):
        approx = sum(w[j] * _peval(A, s[j]) / (z - s[j]) for j in range(N))
        exact = _peval(A, z) / (1.0 + ((z - c) / R) ** N)
        assert np.abs(approx - exact).max() <= 1e-13 * np.abs(exact).max()


def test_moments_are_taylor_coefficients_for_polynomials():
    """sum_j w_j (s_j - c)^{-p} T(s_j) = -T^{(p-1)}(c)/(p-1)! exactly for deg T <= N+p-2."""
    rng = np.random.Generator(np.random.PCG64(2))
    c, R, N, P = 0.5 + 0.5j, 1.3, 12, 4
    s, w = M.circle_nodes(c, R, N)
    W = M.moment_weights(s, w, c, P)
    for p in range(1, P + 1):
        A = _poly_matrix(rng, N + p - 2)
        mom = sum(W[j, p - 1] * _peval(A, s[j]) for j in range(N))
        ref = -_peval(A, c, deriv=p - 1) / math.factorial(p - 1)
        assert np.abs(mom - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


def test_rational_closed_form():
    """sum_j 1/(s_j - x) over the unit-circle nodes s_j = e^{i(theta0 + 2 pi j/N)} equals
    -N x^{N-1}/(x^N - e^{i N theta0}) (roots of x^N = e^{i N theta0})."""
    N = 20
    s, _ = M.circle_nodes(0.0, 1.0, N)
    theta0 = np.pi / N
    for x in (0.3 + 0.2j, 1.7 - 0.4j, -0.9j):
        lhs = np.sum(1.0 / (s - x))
        rhs = -N * x ** (N - 1) / (x ** N - np.exp(1j * N * theta0))
        assert abs(lhs - rhs) < 1e-14 * np.sum(np.abs(1.0 / (s - x)))


@pytest.fixture(scope="module")
def sphere1():
    xyz, tri = synth.icosphere(1)
    return M.Operator(xyz, tri)


def test_bem_moments_equal_derivatives(sphere1):
    """For the BEM kernel the p-th contour moment is -T^{(p-1)}(c) V/(p-1)! up to an
    aliasing error ~ (R r_max)^N / N! (about 1e-21 here)."""
    op = sphere1
    V = synth.probe_block(op.n, 3, seed=4)
    c, R, N, P = 4.0, 1.5, 32, 3
    s, w = M.circle_nodes(c, R, N)
    W = M.moment_weights(s, w, c, P)
    mom = M.contour_moments(op, s, W, V)
    for p in range(1, P + 1):
        ref = -op.apply(c, V, deriv=p - 1) / math.factorial(p - 1)
        assert np.linalg.norm(mom[p - 1] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_cheb_rule_exact_on_polynomials():
    rng = np.random.Generator(np.random.PCG64(3))
    a, b, N = 2.0, 8.0, 10
    kappa, coef = M.cheb_nodes(a, b, N)
    xi = (kappa - 0.5 * (a + b)) / (0.5 * (b - a))
    assert np.allclose(np.sort(xi), np.sort(np.polynomial.chebyshev.chebpts1(N)), atol=1e-15)
    pw = rng.standard_normal(N)  # power-basis coefficients in xi, degree N-1
    samples = np.polynomial.polynomial.polyval(xi, pw)
    ref = np.polynomial.chebyshev.poly2cheb(pw)
    assert np.allclose(coef @ samples, ref, atol=1e-12 * np.abs(ref).max())
    # and the interpolant reproduces the polynomial anywhere in the interval
    for x in (-0.9, 0.1, 0.77):
        assert abs(M.cheb_eval(coef @ samples, x) - np.polynomial.polynomial.polyval(x, pw)) < 1e-12


def test_cheb_moments_match_jacobi_anger(sphere1):
    """Off-diagonal Chebyshev coefficient blocks of the BEM operator on [a, b] equal
    sum_q A_b w_q eps_l i^l e^{i alpha r} J_l(beta r)/(4 pi r) (Jacobi-Anger expansion)."""
    op = sphere1
    a, b, N = 2.0, 8.0, 48
    L = 12
    C = M.cheb_moments(op, a, b, N, L, np.eye(op.n, dtype=np.complex128))
    from oracle import _clib

    _, cen, qp, qw = _clib.geometry(op.xyz, op.tri)
    alpha, beta = 0.5 * (a + b), 0.5 * (b - a)
    r = np.linalg.norm(cen[:, None, None, :] - qp[None, :, :, :], axis=-1)  # n x n x 7
    off = ~np.eye(op.n, dtype=bool)
    scale = np.abs(C[0][off]).max()
    for l in range(L):
        eps = 1.0 if l == 0 else 2.0
        with np.errstate(invalid="ignore", divide="ignore"):  # r = 0 only on the diagonal
            ref = np.sum(qw[None, :, :] * eps * (1j ** l) * np.exp(1j * alpha * r)
                         * jv(l, beta * r) / (4 * np.pi * r), axis=-1)
        assert np.abs(C[l][off] - ref[off]).max() <= 1e-13 * scale, l


def test_projection_pins(sphere1):
    op = sphere1
    s, _ = M.circle_nodes(4.0, 1.5, 4)
    P = M.rr_project(op, s, np.eye(op.n))
    for j in range(4):
        assert np.array_equal(P[j], op.dense(s[j]))
    Q, _ = np.linalg.qr(synth.probe_block(op.n, op.n, seed=5))
    Pq = M.rr_project(op, s[:2], Q)
    for j in range(2):
        assert abs(np.linalg.norm(Pq[j]) - np.linalg.norm(op.dense(s[j]))) < 1e-13 * np.linalg.norm(Pq[j])


def test_cauchy_pencil_recovers_polynomial_eigenvalues():
    rng = np.random.Generator(np.random.PCG64(6))
    c, R, N, n = 0.0, 1.0, 24, 6
    lam = np.array([0.2 + 0.1j, -0.5j, 0.6, 1.8, -2.5 + 0.3j, 3.0j])  # 3 inside, 3 outside
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = X @ np.diag(lam) @ np.linalg.inv(X)
    s, w = M.circle_nodes(c, R, N)
    Bs = [w[j] * (A - s[j] * np.eye(n)) for j in range(N)]
    inside, _, _, _ = M.solve_cauchy_reduced(Bs, s, c, R)
    assert np.allclose(np.sort_complex(inside), np.sort_complex(lam[np.abs(lam) < 1]), atol=1e-12)
    # quadratic T(z) = z^2 I + z C1 + C0: eigenvalues from the companion pencil
    C1 = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    C0 = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    comp = np.block([[np.zeros((n, n)), np.eye(n)], [-C0, -C1]])
    ev = np.linalg.eigvals(comp)
    Bs = [w[j] * (s[j] ** 2 * np.eye(n) + s[j] * C1 + C0) for j in range(N)]
    inside, _, _, _ = M.solve_cauchy_reduced(Bs, s, c, R)
    ref = ev[np.abs(ev) < 1]
    assert inside.size == ref.size
    for z in ref:
        assert np.min(np.abs(inside - z)) < 1e-11


def test_cheb_pencil_recovers_polynomial_eigenvalues():
    rng = np.random.Generator(np.random.PCG64(7))
    n, a, b, N = 5, 2.0, 8.0, 12
    lam = np.array([2.5, 3.7, 6.1, 9.0, 1.0])  # three inside [a, b]
    X = rng.standard_normal((n, n))
    A = X @ np.diag(lam) @ np.linalg.inv(X)
    kappa, coef = M.cheb_nodes(a, b, N)
    samples = [A - k * np.eye(n) for k in kappa]
    Bs = [sum(coef[l, k] * samples[k] for k in range(N)) for l in range(N)]
    # the interpolant of a degree-1 function: higher coefficients vanish
    assert max(np.abs(Bs[l]).max() for l in range(2, N)) < 1e-13
    # a degree-3 polynomial eigenproblem keeps every coefficient non-zero
    E2 = 0.05 * rng.standard_normal((n, n))
    E3 = 0.01 * rng.standard_normal((n, n))
    T = lambda k: A - k * np.eye(n) + E2 * (k - 5) ** 2 + E3 * (k - 5) ** 3  # noqa: E731
    Bs = [sum(coef[l, k] * T(kappa[k]) for k in range(N)) for l in range(N)]
    found, Y, _, _ = M.solve_cheb_reduced(Bs, a, b)
    assert found.size >= 1
    for k, y in zip(found, Y.T):
        smin = np.linalg.svd(T(k), compute_uv=False)[-1]
        assert smin < 1e-12 * np.linalg.norm(T(k))
        assert np.linalg.norm(T(k) @ y) < 1e-11 * np.linalg.norm(T(k))


def test_inverse_power_step_equals_dense_shift_invert():
    rng = np.random.Generator(np.random.PCG64(8))
    n, N, shift = 5, 6, 0.3 + 0.1j
    s, w = M.circle_nodes(0.2, 1.0, N)
    Bs = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(N)]
    A, Mm = M.cauchy_pencil(Bs, s)
    v = [rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2)) for _ in range(N)]
    u = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    wv = np.vstack(v + [u])
    ref = np.linalg.solve(A - shift * Mm, Mm @ wv)
    v2, u2 = M.inverse_power_step(Bs, s, shift, v, u)
    got = np.vstack(v2 + [u2])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d", [5, 6])
@pytest.mark.parametrize("shift", [0.0, 0.3 + 0.1j])
def test_cheb_inverse_power_step_equals_dense_shift_invert(d, shift):
    """One step of Algorithm 2 by block elimination equals (A - s M)^{-1} M w for the
    Chebyshev linearisation, for both parities of the degree d."""
    rng = np.random.Generator(np.random.PCG64(9 + d))
    n = 4
    Bs = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(d + 1)]
    A, Mm = M.cheb_pencil(Bs)
    v = [rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2)) for _ in range(d)]
    ref = np.linalg.solve(A - shift * Mm, Mm @ np.vstack(v))
    got = np.vstack(M.cheb_inverse_power_step(Bs, shift, v))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_interval_iteration_matches_contour_iteration(sphere1):
    """n = 80: the Chebyshev route (Algorithm 2 in Algorithm 3, pencil eq. sc1_chebyshev_red)
    on [2.5, 5] finds the same four eigenvalues as the Cauchy route on |z - 4| < 1.5, each
    with residual <= 1e-12; the two share only the operator."""
    op = sphere1
    V = synth.probe_block(op.n, 8, seed=1)
    lc, _, rc, _, _ = M.subspace_iteration(op, 4.0, 1.5, 32, V, q=10, tol=1e-12)
    li, _, ri, _, _ = M.cheb_subspace_iteration(op, 2.5, 5.0, 24, V, q=10, tol=1e-12, imag_tol=1e-2)
    assert ri.max() <= 1e-12 and li.size == lc.size == 4
    assert np.abs(np.sort_complex(li) - np.sort_complex(lc)).max() <= 1e-10 * np.abs(lc).max()


def test_end_to_end_small_sphere_vs_brute_force(sphere1):
    """n = 80: Rayleigh-Ritz eigenvalues inside |z - 4| < 1.5 (N = 32) agree with MSLP on
    det T to ~1e-12 and their number with the argument principle."""
    op = sphere1
    V = synth.probe_block(op.n, 8, seed=1)
    lam, X, res, outer, _ = M.subspace_iteration(op, 4.0, 1.5, 32, V, q=10, tol=1e-12)
    assert res.max() <= 1e-12
    cnt = M.argument_count(op, 4.0, 1.5, nodes=96)
    assert abs(cnt - round(cnt.real)) < 1e-8 and lam.size == round(cnt.real) == 4
    for l0 in lam:
        assert abs(M.mslp(op, l0) - l0) < 1e-12 * abs(l0)
    # the triple near 4.49 is exactly degenerate on the icosahedral mesh
    assert np.abs(lam[1:] - lam[1]).max() < 1e-10


def test_sphere_eigenvalues_approach_table2():
    """Eigenvalues of the discrete operator near pi and 4.4934 (Table 2) approach the
    zeros of j_0 and j_1 at second order in the mesh size."""
    tab = np.loadtxt(os.path.join(GOLDEN, "sphere_dirichlet_eigs.txt"))
    j0 = brentq(lambda x: spherical_jn(0, x), 3.0, 3.3)
    j1 = brentq(lambda x: spherical_jn(1, x), 4.3, 4.6)
    assert abs(tab[0, 0] - j0) < 1e-4 and abs(tab[1, 0] - j1) < 1e-4
    errs = []
    for L in (1, 2):
        xyz, tri = synth.icosphere(L)
        op = M.Operator(xyz, tri)
        V = synth.probe_block(op.n, 8, seed=1)
        lam, _, res, _, _ = M.subspace_iteration(op, 4.0, 1.5, 32, V, q=10, tol=1e-12)
        assert lam.size == 4 and res.max() <= 1e-12
        errs.append([abs(lam[0] - j0), abs(lam[1] - j1)])
    errs = np.array(errs)
    assert np.all(errs[1] < 0.07) and np.all(3.0 < errs[0] / errs[1]) and np.all(errs[0] / errs[1] < 5.0)


def test_golden_tables_match_closed_forms():
    """Table 2 values are zeros of spherical Bessel functions j_l with multiplicity 2l+1;
    Table 1 values are pi sqrt(n1^2+n2^2+n3^2), n_i >= 1 (the reading of eq. cubeev that
    reproduces the table)."""
    sph = np.loadtxt(os.path.join(GOLDEN, "sphere_dirichlet_eigs.txt"))
    zeros = []
    for l in range(5):
        grid = np.linspace(0.5, 8.5, 4001)
        f = spherical_jn(l, grid)
        for i in np.flatnonzero(np.sign(f[:-1]) != np.sign(f[1:])):
            zeros.append((brentq(lambda x: spherical_jn(l, x), grid[i], grid[i + 1]), 2 * l + 1))
    zeros.sort()
    for (val, mult), (z, mz) in zip(sph, zeros[: len(sph)]):
        # the table is printed to four decimals, some truncated (6.2831 for 2 pi)
        assert abs(val - z) < 1e-4 and mult == mz
    cube = np.loadtxt(os.path.join(GOLDEN, "cube_dirichlet_eigs.txt"))
    ks = {}
    for n1 in range(1, 5):
        for n2 in range(1, 5):
            for n3 in range(1, 5):
                k = round(np.pi * np.sqrt(n1 * n1 + n2 * n2 + n3 * n3), 6)
                ks[k] = ks.get(k, 0) + 1
    ref = sorted(ks.items())[: len(cube)]
    for (val, mult), (k, mk) in zip(cube, ref):
        assert abs(val - k) < 1.5e-6 and mult == mk
