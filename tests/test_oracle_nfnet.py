"""Pins of the oracle's reference of the learned near-field network (oracle/nfnet.py), CPU only:
back-propagation against central finite differences of the loss, the forward pass against
closed forms, Adam's first step against its closed form, the input map against rigid-motion,
scaling, vertex-order and reflection invariances and a hand-computed case, Radon's points
against the rule of the oracle's C core, and the output map against its inverse."""
import numpy as np
import pytest

from oracle import _clib
from oracle import nfnet as O


def _params(seed, scale=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal(O.N_PARAMS) * scale
    W1 = O.split(p)[0]
    W1[:, O.F:] = 0.0
    return p


def test_backward_matches_finite_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    p = _params(2)
    X = rng.standard_normal((7, O.F))
    T = rng.standard_normal((7, O.O))
    _, g = O.loss_grad(p, X, T)
    W1 = O.split(np.arange(O.N_PARAMS))[0]
    used = np.setdiff1d(np.arange(O.N_PARAMS), W1[:, O.F:].ravel())
    idx = rng.choice(used, 300, replace=False)
    # every block represented: the last biases and output weights too
    idx = np.unique(np.concatenate([idx, np.arange(O.N_PARAMS - 300, O.N_PARAMS)]))
    eps = 1e-6
    for i in idx:
        e = np.zeros(O.N_PARAMS)
        e[i] = eps
        fd = (O.loss(p + e, X, T) - O.loss(p - e, X, T)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    # padded input columns get no gradient
    assert np.all(g[W1[:, O.F:].ravel()] == 0.0)


def test_forward_closed_forms():
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((5, O.F))
    p = np.zeros(O.N_PARAMS)
    W1, b1, W2, b2, W3, b3, W4, b4 = O.split(p)
    b4[:] = [0.25, -1.5]
    assert np.allclose(O.forward(p, X), [[0.25, -1.5]] * 5, rtol=0, atol=0)
    # one path: y0 = 2 tanh(tanh(tanh(a x3 + c) - 0.5) + 0.1) + b4_0
    a, c = 0.7, 0.2
    W1[5, 3] = a
    b1[5] = c
    W2[9, 5] = 1.0
    b2[9] = -0.5
    W3[0, 9] = 1.0
    b3[0] = 0.1
    W4[0, 0] = 2.0
    y = O.forward(p, X)
    ref = 2.0 * np.tanh(np.tanh(np.tanh(a * X[:, 3] + c) - 0.5) + 0.1) + 0.25
    assert np.allclose(y[:, 0], ref, rtol=1e-15, atol=1e-15)
    assert np.allclose(y[:, 1], -1.5, rtol=0, atol=0)


def test_adam_first_step_closed_form():
    rng = np.random.Generator(np.random.PCG64(4))
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = O.adam(p, g, np.zeros(50), np.zeros(50), 1, 1e-2)
    # first step: m^ = g, v^ = g^2, so the update is lr g / (|g| + eps)
    assert np.allclose(new, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _rotation(rng):
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return q if np.linalg.det(q) > 0 else -q


def test_features_invariances():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(20):
        P = rng.standard_normal((3, 3))
        x = P.mean(0) + rng.standard_normal(3)
        k = complex(rng.uniform(0.5, 3), rng.uniform(-0.5, 0.5))
        f, h, r0, kh = O.features(P, x, k)
        # rigid motion and scaling (kappa scaled inversely: same kappa h)
        R, t, s = _rotation(rng), rng.standard_normal(3), rng.uniform(0.1, 10.0)
        f2, h2, r02, kh2 = O.features(s * P @ R.T + t, s * R @ x + t, k / s)
        assert np.allclose(f2, f, rtol=1e-12, atol=1e-12) and abs(h2 - s * h) <= 1e-12 * s * h
        assert abs(kh2 - kh) <= 1e-12 * abs(kh)
        # cyclic relabelling and reversed orientation of the vertices
        for order in ([1, 2, 0], [2, 0, 1], [0, 2, 1], [2, 1, 0]):
            assert np.allclose(O.features(P[order], x, k)[0], f, rtol=1e-12, atol=1e-12), order
        # the target mirrored through the triangle's plane
        n = np.cross(P[1] - P[0], P[2] - P[0])
        n /= np.linalg.norm(n)
        xm = x - 2.0 * np.dot(x - P[0], n) * n
        assert np.allclose(O.features(P, xm, k)[0], f, rtol=1e-12, atol=1e-12)


def test_features_hand_computed():
    # equilateral triangle of side 2 in the plane z = 0, target 1 above the centroid
    P = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [1.0, np.sqrt(3.0), 0.0]])
    x = np.array([1.0, np.sqrt(3.0) / 3.0, 1.0])
    f, h, r0, kh = O.features(P, x, 0.25 + 0.05j)
    assert h == 2.0 and abs(r0 - 0.5) < 1e-15 and abs(kh - (0.5 + 0.1j)) < 1e-15
    p, q, u, v, w = 0.5, np.sqrt(3.0) / 2.0, 0.5, np.sqrt(3.0) / 6.0, 0.5
    s = np.sqrt(1.0 / 3.0 + 0.25)  # distance to each vertex, unit frame
    ref = [(p - 0.25) / 0.25, (q - 0.5) / 0.4, (u - 0.5) / 1.5, (v - 0.3) / 1.5, w, 0.0, 0.1 / 0.3, -0.5, 1.0]
    assert np.allclose(f[:9], ref, rtol=0, atol=1e-15)
    assert abs(f[9] - 0.3 / 0.5) < 1e-15  # the centroid point lies straight below
    assert np.allclose(f[16:], 0.5 / s, rtol=1e-15)


def test_radon_points_match_the_c_rule():
    p, q = 0.3, 0.7
    pts = O.radon_points_canonical(p, q)
    bary, w = _clib.radon7()
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [p, q, 0.0]])
    ref = bary @ V
    d = np.linalg.norm(pts[:, None, :] - ref[None, :, :], axis=2)
    assert d.min(axis=1).max() < 1e-15 and len(set(d.argmin(axis=1))) == 7


def test_output_map_round_trip():
    rng = np.random.Generator(np.random.PCG64(6))
    p = _params(7)
    S = (2e-3, 5e-4)
    P = rng.standard_normal((3, 3))
    x = P.mean(0) + 0.5 * rng.standard_normal(3)
    k = 1.3 - 0.2j
    dT = O.correction(p, S, P, x, k)
    t = O.target(P, x, k, dT)
    y = O.forward(p, O.features(P, x, k)[0])[0]
    assert abs(t - (S[0] * y[0] + 1j * S[1] * y[1])) <= 1e-14 * abs(t)


def test_planted_mistakes_are_caught():
    """A wrong tanh derivative or a dropped bias gradient fails the finite-difference pin."""
    rng = np.random.Generator(np.random.PCG64(8))
    p = _params(9)
    X = rng.standard_normal((4, O.F))
    T = rng.standard_normal((4, O.O))
    _, g = O.loss_grad(p, X, T)
    orig = O.backward

    def bad(params, acts, dY):
        out = orig(params, acts, dY)
        out[O.H * O.F_PAD:O.H * O.F_PAD + O.H] = 0.0  # b1's gradient dropped
        return out

    O.backward = bad
    try:
        _, gb = O.loss_grad(p, X, T)
    finally:
        O.backward = orig
    i = O.H * O.F_PAD + int(np.argmax(np.abs(g[O.H * O.F_PAD:O.H * O.F_PAD + O.H])))
    e = np.zeros(O.N_PARAMS)
    e[i] = 1e-6
    fd = (O.loss(p + e, X, T) - O.loss(p - e, X, T)) / 2e-6
    assert abs(fd - gb[i]) > 1e-3 * abs(fd)
