"""Pins of the oracle's quadrature, geometry and self term against closed forms and
independent quadratures (CPU only)."""
from math import factorial

import numpy as np
import pytest

import synth


def test_radon_rule_degree_five(oracle_lib):
    C = oracle_lib._clib
    bary, w = C.radon7()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(bary > 0) and np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    P = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    pts = bary @ P
    for deg in range(7):
        worst = 0.0
        for i in range(deg + 1):
            j = deg - i
            exact = factorial(i) * factorial(j) / factorial(i + j + 2)
            rule = 0.5 * np.sum(w * pts[:, 0] ** i * pts[:, 1] ** j)
            worst = max(worst, abs(rule - exact))
        if deg <= 5:
            assert worst < 1e-15, (deg, worst)
        else:
            assert worst > 1e-6, "a degree-5 rule must not integrate degree 6 exactly"


def test_gauss_legendre_exactness(oracle_lib):
    x, w = oracle_lib._clib.gauss_legendre(12)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(24):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    xr, wr = np.polynomial.legendre.leggauss(12)
    assert np.allclose(np.sort(x), xr, atol=1e-15) and np.allclose(w[np.argsort(x)], wr, atol=1e-14)


def test_icosphere_counts_and_closure():
    prev = 0.0
    for L in range(5):
        xyz, tri = synth.icosphere(L)
        assert xyz.shape == (10 * 4 ** L + 2, 3)
        assert tri.shape == (20 * 4 ** L, 3)
        assert synth.mesh_edges_ok(tri)
        assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0, atol=1e-15)
        p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
        area = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1).sum()
        assert prev < area < 4 * np.pi
        prev = area
    assert 4 * np.pi - prev < 0.02


def test_oracle_geometry_matches_definition(oracle_lib):
    xyz, tri = synth.perturbed_icosphere(1, 0.2, seed=7)
    area, cen, qp, qw = oracle_lib._clib.geometry(xyz, tri)
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    assert np.allclose(area, 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1), rtol=1e-14)
    assert np.allclose(cen, (p0 + p1 + p2) / 3.0, atol=1e-15)
    assert np.allclose(qw.sum(axis=1), area, rtol=1e-14)
    # the centroid is the first quadrature point; all points lie in the triangle's plane
    assert np.allclose(qp[:, 0, :], cen, atol=1e-15)
    nrm = np.cross(p1 - p0, p2 - p0)
    assert np.max(np.abs(np.einsum("nqc,nc->nq", qp - p0[:, None, :], nrm))) < 1e-15


def test_degenerate_triangle_rejected(oracle_lib):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], dtype=float)
    tri = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle_lib._clib.geometry(xyz, tri)
    with pytest.raises(ValueError):
        oracle_lib._clib.geometry(xyz, np.array([[0, 1, 9]], dtype=np.int32))


def _random_triangles(seed, count=6):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        P = rng.standard_normal((3, 3)) * 0.3
        e1, e2 = P[1] - P[0], P[2] - P[0]
        A = 0.5 * np.linalg.norm(np.cross(e1, e2))
        # keep reasonably shaped triangles (smallest angle > 15 degrees)
        ang = []
        for i in range(3):
            a, b = P[(i + 1) % 3] - P[i], P[(i + 2) % 3] - P[i]
            ang.append(np.degrees(np.arccos(a @ b / np.linalg.norm(a) / np.linalg.norm(b))))
        if A > 1e-3 and min(ang) > 15:
            out.append(P)
    return out


def _laplace_edges(P):
    """(1/4 pi) int dA/|x - y| over the triangle, x = centroid, by the edge formula
    sum_e d_e [asinh(l+/d_e) - asinh(l-/d_e)]."""
    x = P.mean(axis=0)
    tot = 0.0
    for e in range(3):
        A, B = P[e], P[(e + 1) % 3]
        t = (B - A) / np.linalg.norm(B - A)
        foot = A + ((x - A) @ t) * t
        d = np.linalg.norm(x - foot)
        lm, lp = (A - foot) @ t, (B - foot) @ t
        tot += d * (np.arcsinh(lp / d) - np.arcsinh(lm / d))
    return tot / (4 * np.pi)


def _duffy(P, kappa, order=64):
    """Independent 2-D reference: split the triangle at the centroid x into three
    triangles (x, P_e, P_e+1); map each from the unit square by
    y = x + u (P_e - x) + u v (P_e+1 - P_e) (Duffy), which cancels the 1/r singularity,
    and integrate exp(i k r)/(4 pi r) with a tensor Gauss-Legendre rule."""
    g, w = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    x = P.mean(axis=0)
    tot = 0.0j
    for e in range(3):
        A, B = P[e], P[(e + 1) % 3]
        jac0 = np.linalg.norm(np.cross(A - x, B - A))
        for vi, wv in zip(g, w):
            dvec = (A - x) + vi * (B - A)
            rho = np.linalg.norm(dvec)
            r = g * rho  # distance at each u
            # integrand * Jacobian (u * jac0) with 1/r = 1/(u rho)
            f = np.exp(1j * kappa * r) / (4 * np.pi * rho) * jac0
            tot += wv * np.sum(w * f)
    return tot


def test_self_term_laplace_limit(oracle_lib):
    C = oracle_lib._clib
    for P in _random_triangles(11):
        assert abs(C.self_term_tri(P, 0.0) - _laplace_edges(P)) < 1e-15 * 10
    s = 0.37
    Pq = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * np.sqrt(3) / 2, 0]])
    exact = np.sqrt(3) * s * np.arcsinh(np.sqrt(3)) / (4 * np.pi)
    assert abs(C.self_term_tri(Pq, 0.0) - exact) < 2e-16 * 4


@pytest.mark.parametrize("kappa", [5 - 1j, 3.0, 7.5 + 0.8j, 0.3])
def test_self_term_complex_kappa_vs_duffy(oracle_lib, kappa):
    C = oracle_lib._clib
    for P in _random_triangles(23, 4):
        ref = _duffy(P, kappa)
        val = C.self_term_tri(P, kappa)
        assert abs(val - ref) <= 5e-15 * abs(ref), (val, ref)


def test_self_term_derivatives(oracle_lib):
    C = oracle_lib._clib
    for P in _random_triangles(5, 3):
        A = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        # d/dk int exp(ikr)/(4 pi r) dA at k = 0 is i A/(4 pi)
        assert abs(C.self_term_tri(P, 0.0, deriv=1) - 1j * A / (4 * np.pi)) < 1e-16
        # derivative order d against a Cauchy-integral derivative of the order-0 value
        k0, rad, M = 4.0 - 0.3j, 0.5, 64
        th = 2 * np.pi * np.arange(M) / M
        vals = np.array([C.self_term_tri(P, k0 + rad * np.exp(1j * t)) for t in th])
        for d in (1, 2, 3):
            fac = float(np.prod(np.arange(1, d + 1)))
            ref = fac * np.mean(vals * np.exp(-1j * d * th)) / rad ** d
            got = C.self_term_tri(P, k0, deriv=d)
            # roundoff of the reference scales with max|T| d!/rad^d
            assert abs(got - ref) <= 1e-13 * np.abs(vals).max() * fac / rad ** d, (d, got, ref)


def test_box_surface_mesh():
    """The box meshes: 4 (nx ny + nx nz + ny nz) triangles, every edge in exactly two faces,
    Euler characteristic 2, total area 2 (ab + ac + bc), all triangles of the grid's size."""
    for dims, counts in (((1.0, 0.8, 0.6), (10, 8, 6)), ((1.0, 0.8, 0.6), (126, 101, 76)), ((2.0, 1.0, 0.5), (3, 2, 1))):
        xyz, tri = synth.box_surface(dims, counts)
        nx, ny, nz = counts
        a, b, c = dims
        assert tri.shape[0] == 4 * (nx * ny + nx * nz + ny * nz)
        assert synth.mesh_edges_ok(tri)
        assert xyz.shape[0] - tri.shape[0] * 3 // 2 + tri.shape[0] == 2
        P = xyz[tri]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        assert abs(area.sum() - 2 * (a * b + a * c + b * c)) < 1e-10
        assert np.all(area > 0)
        # every vertex lies on the box surface
        on = np.isclose(xyz[:, 0], 0) | np.isclose(xyz[:, 0], a) | np.isclose(xyz[:, 1], 0) | \
            np.isclose(xyz[:, 1], b) | np.isclose(xyz[:, 2], 0) | np.isclose(xyz[:, 2], c)
        assert on.all()


def test_geodesic_sphere_mesh():
    """Class-I geodesic spheres: 20 f^2 triangles and 10 f^2 + 2 vertices, closed, every
    vertex on the unit sphere, every triangle oriented outward; f = 1 is the icosahedron
    and f = 2 has exactly the vertex set of the once-split icosphere (the midpoints of flat
    edges projected); the enclosed volume (divergence theorem) grows toward 4 pi / 3."""
    vols = []
    for f in (1, 2, 3, 5, 12):
        xyz, tri = synth.geodesic_sphere(f)
        assert tri.shape == (20 * f * f, 3) and xyz.shape == (10 * f * f + 2, 3)
        assert synth.mesh_edges_ok(tri)
        assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0, atol=1e-14)
        P = xyz[tri]
        nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        assert np.all((nrm * P.mean(axis=1)).sum(axis=1) > 0)
        vols.append((nrm * P[:, 0]).sum() / 6.0)
    assert np.all(np.diff(vols) > 0) and vols[-1] < 4 * np.pi / 3 and vols[-1] > 0.99 * 4 * np.pi / 3
    x1, t1 = synth.icosahedron()
    xg, tg = synth.geodesic_sphere(1)
    assert np.array_equal(np.sort(np.round(xg, 13), axis=0), np.sort(np.round(x1, 13), axis=0))
    xi, _ = synth.icosphere(1)
    x2, _ = synth.geodesic_sphere(2)
    assert np.array_equal(np.sort(np.round(x2, 12), axis=0), np.sort(np.round(xi, 12), axis=0))


def test_ellipsoid_batch_recipe():
    """The seeded ellipsoid batch: deterministic, 20 f^2 triangles with f in [10, 44],
    semi-axes in [0.5, 1.5] (the vertices satisfy the ellipsoid's equation), centres in
    [3, 7]; a small batch is checked here, the 64-mesh default only for its size range."""
    a = synth.ellipsoid_batch(count=3, seed=4, freq=(2, 5))
    b = synth.ellipsoid_batch(count=3, seed=4, freq=(2, 5))
    for (xa, ta, axa, ca), (xb, tb, axb, cb) in zip(a, b):
        assert np.array_equal(xa, xb) and np.array_equal(ta, tb) and ca == cb
        f = int(round((ta.shape[0] / 20) ** 0.5))
        assert 2 <= f <= 5 and ta.shape[0] == 20 * f * f
        assert np.all((axa >= 0.5) & (axa <= 1.5)) and 3.0 <= ca <= 7.0
        assert np.allclose(((xa / axa[None, :]) ** 2).sum(axis=1), 1.0, atol=1e-13)
        assert synth.mesh_edges_ok(ta)


def test_harmonic_sphere_shape():
    """20 f^2 triangles, closed (every edge in two faces), radius within 1 +- 0.1 sum |c Y|,
    seeded (same seed, same mesh) and star-shaped around the origin."""
    import synth

    xyz, tri = synth.harmonic_sphere(9, seed=5)
    assert tri.shape == (20 * 81, 3) and xyz.shape == (10 * 81 + 2, 3)
    assert synth.mesh_edges_ok(tri)
    r = np.linalg.norm(xyz, axis=1)
    assert 0.8 < r.min() < 1.0 < r.max() < 1.2
    xyz2, tri2 = synth.harmonic_sphere(9, seed=5)
    assert np.array_equal(xyz, xyz2) and np.array_equal(tri, tri2)
    P = xyz[tri]
    vol6 = np.einsum("ij,ij->i", P[:, 0], np.cross(P[:, 1], P[:, 2]))
    assert (vol6 > 0).all()  # every face sees the origin on the same side
