"""Pins of the oracle's near-field quadrature (adaptive cubature of the Green's function over
a triangle, Section 1, eq. GreenFun) and of its near-pair list, against results fixed
independently of it:

* kappa = 0: the closed form of the potential of a uniform flat triangle (Wilton, Rao,
  Glisson, Arvas, Butler and Glisson, IEEE Trans. Antennas Propag. 32 (1984)), written here
  in a cancellation-free form;
* complex kappa: that closed form plus the integral of the smooth remainder
  (e^{i kappa R} - 1)/(4 pi R) by a composite collapsed Gauss product rule on a uniform
  subdivision (no adaptivity);
* far from the triangle the integral agrees with Radon's 7-point rule to its
  degree-5 error;
* the near-pair list equals a vectorised brute-force evaluation of its definition.
"""
import numpy as np
import pytest


def _wilton(x, P):
    """int over triangle P of 1/(4 pi |x - y|) dA_y in closed form."""
    P = np.asarray(P, dtype=np.float64).reshape(3, 3)
    nrm = np.cross(P[1] - P[0], P[2] - P[0])
    nrm /= np.linalg.norm(nrm)
    d = float(np.dot(x - P[0], nrm))
    xp = x - d * nrm
    total = 0.0
    for e in range(3):
        A, B = P[e], P[(e + 1) % 3]
        t = (B - A) / np.linalg.norm(B - A)
        u = np.cross(t, nrm)
        p = float(np.dot(A - xp, u))
        sA, sB = float(np.dot(A - xp, t)), float(np.dot(B - xp, t))
        R0sq = p * p + d * d
        if R0sq == 0.0:
            continue
        RA, RB = np.sqrt(R0sq + sA * sA), np.sqrt(R0sq + sB * sB)

        def f(R, s):  # R + s without cancellation ((R + s)(R - s) = R0^2)
            return R + s if s >= 0 else R0sq / (R - s)

        total += p * np.log(f(RB, sB) / f(RA, sA))
        total -= abs(d) * (np.arctan2(p * sB, R0sq + abs(d) * RB) - np.arctan2(p * sA, R0sq + abs(d) * RA))
    return total / (4.0 * np.pi)


def _split(P, levels):
    """The 4**levels congruent midpoint subtriangles of P, as an array (count, 3, 3)."""
    T = np.asarray(P, dtype=np.float64).reshape(1, 3, 3)
    for _ in range(levels):
        m01, m12, m20 = (T[:, 0] + T[:, 1]) / 2, (T[:, 1] + T[:, 2]) / 2, (T[:, 2] + T[:, 0]) / 2
        T = np.concatenate([np.stack([T[:, 0], m01, m20], 1), np.stack([m01, T[:, 1], m12], 1),
                            np.stack([m20, m12, T[:, 2]], 1), np.stack([m01, m12, m20], 1)])
    return T


def _smooth_remainder(x, P, kappa, levels=5, order=16):
    """int over P of (e^{i kappa R} - 1)/(4 pi R) dA: a collapsed order x order Gauss product
    rule on each of the 4**levels midpoint subtriangles (the integrand is smooth, with a
    kink of R only at the foot of x, so the composite rule converges quickly)."""
    T = _split(P, levels)
    g, w = np.polynomial.legendre.leggauss(order)
    u = 0.5 * (1 + g)
    U, Vv = np.meshgrid(u, u, indexing="ij")
    Wt = (np.outer(0.5 * w, 0.5 * w) * U).ravel()
    s, t = (U * (1 - Vv)).ravel(), (U * Vv).ravel()
    e1, e2 = T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]
    twoA = np.linalg.norm(np.cross(e1, e2), axis=1)
    y = T[:, None, 0] + s[None, :, None] * e1[:, None] + t[None, :, None] * e2[:, None]
    R = np.linalg.norm(x[None, None, :] - y, axis=-1)
    w_ = kappa * R
    # (e^{iw} - 1)/R, series for small |w| to avoid cancellation
    f = np.where(np.abs(w_) < 1e-3, 1j * kappa * (1 + 0.5j * w_ - w_ * w_ / 6), np.expm1(1j * w_) / R)
    return np.sum(twoA[:, None] * Wt[None, :] * f) / (4.0 * np.pi)


def _cases(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        P = rng.normal(size=(3, 3))
        h = max(np.linalg.norm(P[j] - P[(j + 1) % 3]) for j in range(3))
        x = P.mean(0) + rng.normal(size=3) * h * [0.1, 0.4, 1.0, 2.0][i % 4]
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        nrm /= np.linalg.norm(nrm)
        if i % 5 == 0:  # in the plane of the triangle, outside it
            x = x - np.dot(x - P[0], nrm) * nrm
            bary = np.linalg.lstsq(np.stack([P[1] - P[0], P[2] - P[0]], 1), x - P[0], rcond=None)[0]
            if bary.min() > 0 and bary.sum() < 1:
                x = x + 2.0 * (x - P.mean(0)) + 1.5 * (P[1] - P[0])
        if i % 7 == 3:  # close to an edge line, off the triangle
            x = P[0] + (P[1] - P[0]) * rng.uniform(1.2, 1.8) + nrm * 1e-6 * h
        out.append((x, P, h))
    return out


def test_laplace_matches_closed_form(oracle_lib):
    from oracle import _clib

    worst = 0.0
    for x, P, _ in _cases(11, 40):
        v = _clib.tri_integral(x, P, [0.0])[0]
        ref = _wilton(x, P)
        assert abs(v.imag) <= 1e-15 * abs(ref)
        worst = max(worst, abs(v - ref) / abs(ref))
    assert worst <= 1e-13, worst


def test_helmholtz_matches_closed_form_plus_smooth_part(oracle_lib):
    from oracle import _clib

    worst = 0.0
    for x, P, h in _cases(12, 24):
        ks = np.array([0.5, 1.0 + 0.3j, 2.0 - 0.4j]) / h
        v = _clib.tri_integral(x, P, ks)
        for k, vk in zip(ks, v):
            ref = _wilton(x, P) + _smooth_remainder(x, P, k)
            worst = max(worst, abs(vk - ref) / abs(ref))
    assert worst <= 1e-12, worst


def test_far_field_agrees_with_radon_rule(oracle_lib):
    """At distance D the 7-point rule (degree 5) errs by O((h/D)^6 + (kappa h)^6)."""
    from oracle import _clib

    bary, w = _clib.radon7()
    rng = np.random.default_rng(13)
    for _ in range(8):
        P = rng.normal(size=(3, 3))
        h = max(np.linalg.norm(P[j] - P[(j + 1) % 3]) for j in range(3))
        dirn = rng.normal(size=3)
        x = P.mean(0) + 40.0 * h * dirn / np.linalg.norm(dirn)
        A = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        k = (0.05 + 0.01j) / h
        y = bary @ P
        r = np.linalg.norm(x - y, axis=1)
        seven = np.sum(A * w * np.exp(1j * k * r) / (4 * np.pi * r))
        v = _clib.tri_integral(x, P, [k])[0]
        assert abs(v - seven) <= 1e-8 * abs(v)


def test_subdivision_invariance(oracle_lib):
    """The integral over a triangle equals the sum over the three triangles joining its
    centroid to its edges (a partition the refinement never produces)."""
    from oracle import _clib

    for x, P, h in _cases(14, 12):
        ks = [0.0, (1.0 + 0.5j) / h]
        whole = _clib.tri_integral(x, P, ks)
        g = P.mean(0)
        parts = sum(_clib.tri_integral(x, np.stack([P[e], P[(e + 1) % 3], g]), ks) for e in range(3))
        assert np.max(np.abs(parts - whole) / np.abs(whole)) <= 1e-13


def _near_pairs_brute(xyz, tri, eta):
    P = xyz[tri]
    cen = ((P[:, 0] + P[:, 1]) + P[:, 2]) / 3.0
    h2 = np.zeros(len(tri))
    for e in range(3):
        d = P[:, (e + 1) % 3] - P[:, e]
        h2 = np.maximum(h2, d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    dx = cen[:, None, 0] - cen[None, :, 0]
    dy = cen[:, None, 1] - cen[None, :, 1]
    dz = cen[:, None, 2] - cen[None, :, 2]
    d2 = dx * dx + dy * dy + dz * dz
    near = d2 < (eta * eta) * h2[None, :]
    np.fill_diagonal(near, False)
    rows, cols = np.nonzero(near)
    rowptr = np.zeros(len(tri) + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr), cols.astype(np.int32)


@pytest.mark.parametrize("mesh", ["icosphere2", "box", "ellipsoid"])
def test_near_pairs_match_brute_force(oracle_lib, mesh):
    import synth
    from oracle import _clib

    if mesh == "icosphere2":
        xyz, tri = synth.icosphere(2)
    elif mesh == "box":
        xyz, tri = synth.box_surface((1.0, 0.8, 0.6), (10, 8, 6))
    else:
        xyz, tri = synth.ellipsoid(2, (1.3, 0.9, 0.6))
    for eta in (1.0, 2.0, 3.0):
        rp, col = _clib.near_pairs(xyz, tri, eta)
        rp2, col2 = _near_pairs_brute(xyz, tri, eta)
        assert np.array_equal(rp, rp2) and np.array_equal(col, col2)


def test_correction_is_integral_minus_seven_point(oracle_lib):
    """dT of a pair is the adaptive integral minus the dense operator's 7-point entry."""
    import synth
    from oracle import _clib

    xyz, tri = synth.icosphere(1)
    ks = [2.0, 3.0 + 0.5j]
    rp, col, dT = _clib.nearfield_correction(xyz, tri, 2.0, ks)
    assert col.size > 0
    for j, k in enumerate(ks):
        T = _clib.dense(xyz, tri, k)
        for a in (0, 17, 63):
            for i in range(rp[a], rp[a + 1]):
                b = col[i]
                exact = _clib.tri_integral(xyz[tri[a]].mean(0), xyz[tri[b]], [k])[0]
                assert abs(dT[j, i] - (exact - T[a, b])) <= 1e-15 * abs(exact)


def test_correction_vanishes_beyond_a_few_diameters(oracle_lib):
    """The 7-point rule is accurate away from the source triangle: corrections of pairs
    between 2 and 3 longest edges apart stay below 1e-5 of their entries, at least a hundred
    times below the largest correction within 2 (so eta = 2 captures the part of the operator
    the rule gets wrong)."""
    import synth
    from oracle import _clib

    xyz, tri = synth.icosphere(2)
    k = 3.0 + 0.2j
    rp2, col2 = _clib.near_pairs(xyz, tri, 2.0)
    rp3, col3, dT3 = _clib.nearfield_correction(xyz, tri, 3.0, [k])
    T = _clib.dense(xyz, tri, k)
    inner = set()
    for a in range(len(tri)):
        inner.update((a, int(b)) for b in col2[rp2[a]:rp2[a + 1]])
    outer_worst = inner_worst = 0.0
    for a in range(len(tri)):
        for i in range(rp3[a], rp3[a + 1]):
            rel = abs(dT3[0, i]) / abs(T[a, col3[i]])
            if (a, int(col3[i])) in inner:
                inner_worst = max(inner_worst, rel)
            else:
                outer_worst = max(outer_worst, rel)
    assert 0.0 < outer_worst <= 1e-5, outer_worst
    assert inner_worst >= 100.0 * outer_worst, (inner_worst, outer_worst)


def test_corrected_operator_differs_only_on_near_pairs(oracle_lib):
    from oracle import _clib
    from oracle import method as M
    import synth

    xyz, tri = synth.icosphere(1)
    k = 3.5 + 0.2j
    T = M.Operator(xyz, tri).dense(k)
    Tn = M.Operator(xyz, tri, nearfield_eta=2.0).dense(k)
    rp, col, dT = _clib.nearfield_correction(xyz, tri, 2.0, [k])
    D = np.zeros_like(T)
    D[np.repeat(np.arange(len(tri)), np.diff(rp)), col] = dT[0]
    assert np.array_equal(Tn - T == 0, D == 0)
    assert np.abs((Tn - T) - D).max() <= 1e-17 * np.abs(T).max() * 10
