"""Plain FP64 reference of the learned near-field correction: the map from a (source triangle,
target point, wavenumber) triple to the network's inputs, the network itself (a perceptron with
three hidden layers of 128 tanh units), its loss, its gradients by hand-written
back-propagation, and the Adam update.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It never imports the product package and shares no code with it.

What is learned (not a step of the paper's method: a surrogate for the near-field refinement
of the boundary integral of Section 1, eq. GreenFun): for a near pair, the correction
dT = (integral of g over the source triangle) - (its 7-point value), g(r) = exp(i kappa r)/(4 pi r).

Canonical frame of a source triangle: its longest edge A -> B (the first longest of
P0P1, P1P2, P2P0 in that order) on the x axis, the third vertex C in the upper half plane,
lengths divided by h = |B - A|, so A = (0, 0), B = (1, 0), C = (p, q), q > 0; the target x
has coordinates (u, v, w) (w along the normal (B - A) x (C - A)); when p > 1/2 the frame is
mirrored across u = 1/2 (p -> 1 - p, u -> 1 - u); w enters as |w|.  Scaling the triangle by h
and the wavenumber by 1/h leaves h dT_unit(kappa h), so the unit-frame correction depends on
(p, q, u, v, |w|, kappa h) only.

The 19 inputs (each an affine or reciprocal map of those, fixed here):
  (p - 0.25)/0.25, (q - 0.5)/0.4, (u - 0.5)/1.5, (v - 0.3)/1.5, |w|, 2 Re(kappa h) - 1,
  Im(kappa h)/0.3, r0 - 1, 0.5/r0, 0.3/r_k (k < 7), 0.5/s_k (k < 3)
with r0 the distance of the target to the centroid ((1 + p)/3, q/3, 0), r_k its distance to
the points of Radon's rule listed as: centroid, then the points with barycentric weight
a1 = (9 - 2 sqrt 15)/21 on A, B, C (the others b1 = (6 + sqrt 15)/21), then those with
a2 = (9 + 2 sqrt 15)/21 on A, B, C (the others b2 = (6 - sqrt 15)/21), and s_k its distance to
A, B, C.  The network's two outputs y approximate the scaled correction
    t = 4 pi r0^KPOW dT_unit,    (Re t, Im t) ~ (S_re y_0, S_im y_1)
with output scales S fixed by the training set; dT = h dT_unit.  The factor r0^KPOW takes out
most of the correction's decay with distance (the rule's error falls like r0^-7 far away); dT
is independent of kappa to first order (the rule integrates the linear term of exp(i kappa r)
exactly), so the network's dependence on kappa h is weak.

Parameter vector (the device layout): W1 [128 x 32] (input columns 19..31 unused, zero),
b1 [128], W2 [128 x 128], b2 [128], W3 [128 x 128], b3 [128], W4 [2 x 128], b4 [2]; row-major,
out x in.
"""
from __future__ import annotations

import numpy as np

H = 128        # hidden width
F = 19         # inputs
F_PAD = 32     # input columns in W1
O = 2          # outputs
KPOW = 4       # power of r0 in the scaled target
N_PARAMS = H * F_PAD + H + 2 * (H * H + H) + O * H + O


def split(params):
    """Views (W1, b1, W2, b2, W3, b3, W4, b4) of a parameter vector in the layout above."""
    params = np.asarray(params)
    shapes = [(H, F_PAD), (H,), (H, H), (H,), (H, H), (H,), (O, H), (O,)]
    out, off = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(params[off:off + size].reshape(s))
        off += size
    assert off == N_PARAMS
    return out


def radon_points_canonical(p, q):
    """The 7 points of Radon's rule on the triangle A = (0,0,0), B = (1,0,0), C = (p,q,0), in the
    order of the module docstring (barycentric weights written out from their closed forms)."""
    s15 = np.sqrt(15.0)
    a1, b1 = (9.0 - 2.0 * s15) / 21.0, (6.0 + s15) / 21.0
    a2, b2 = (9.0 + 2.0 * s15) / 21.0, (6.0 - s15) / 21.0
    bary = [(1 / 3, 1 / 3, 1 / 3),
            (a1, b1, b1), (b1, a1, b1), (b1, b1, a1),
            (a2, b2, b2), (b2, a2, b2), (b2, b2, a2)]
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [p, q, 0.0]])
    return np.array([la * V[0] + lb * V[1] + lc * V[2] for la, lb, lc in bary])


def canonical(P, x):
    """(p, q, u, v, |w|, h) of source triangle P (3 x 3 vertices) and target x, per the module
    docstring."""
    P = np.asarray(P, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    lens = [np.linalg.norm(P[(e + 1) % 3] - P[e]) for e in range(3)]
    e = 0
    for k in (1, 2):
        if lens[k] > lens[e]:
            e = k
    A, B, C = P[e], P[(e + 1) % 3], P[(e + 2) % 3]
    h = lens[e]
    ex = (B - A) / h
    nrm = np.cross(B - A, C - A)
    nrm = nrm / np.linalg.norm(nrm)
    ey = np.cross(nrm, ex)
    p, q = np.dot(C - A, ex) / h, np.dot(C - A, ey) / h
    u, v, w = np.dot(x - A, ex) / h, np.dot(x - A, ey) / h, np.dot(x - A, nrm) / h
    if p > 0.5:
        p, u = 1.0 - p, 1.0 - u
    return p, q, u, v, abs(w), h


def features(P, x, kappa):
    """(inputs[19], h, r0, kappa h) of one triple."""
    p, q, u, v, w, h = canonical(P, x)
    kh = complex(kappa) * h
    X = np.array([u, v, w])
    c = np.array([(1.0 + p) / 3.0, q / 3.0, 0.0])
    r0 = np.linalg.norm(X - c)
    rk = np.linalg.norm(X[None, :] - radon_points_canonical(p, q), axis=1)
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [p, q, 0.0]])
    sk = np.linalg.norm(X[None, :] - V, axis=1)
    f = np.concatenate([[(p - 0.25) / 0.25, (q - 0.5) / 0.4, (u - 0.5) / 1.5, (v - 0.3) / 1.5, w,
                         2.0 * kh.real - 1.0, kh.imag / 0.3, r0 - 1.0, 0.5 / r0], 0.3 / rk, 0.5 / sk])
    return f, h, r0, kh


def forward(params, X, keep=False):
    """Outputs Y (B x 2) of inputs X (B x 19 or B x 32); with keep=True also the activations
    [X padded, A1, A2, A3] that back-propagation needs."""
    W1, b1, W2, b2, W3, b3, W4, b4 = split(params)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    Xp = np.zeros((X.shape[0], F_PAD))
    Xp[:, :X.shape[1]] = X
    A1 = np.tanh(Xp @ W1.T + b1)
    A2 = np.tanh(A1 @ W2.T + b2)
    A3 = np.tanh(A2 @ W3.T + b3)
    Y = A3 @ W4.T + b4
    return (Y, [Xp, A1, A2, A3]) if keep else Y


def backward(params, acts, dY):
    """Gradient, in the parameter layout, of sum(dY * Y) (the vector-Jacobian product of the
    network at the kept activations): the chain rule layer by layer, tanh' = 1 - tanh^2."""
    W1, b1, W2, b2, W3, b3, W4, b4 = split(params)
    Xp, A1, A2, A3 = acts
    dY = np.asarray(dY, dtype=np.float64)
    gW4 = dY.T @ A3
    gb4 = dY.sum(0)
    dZ3 = (dY @ W4) * (1.0 - A3 * A3)
    gW3 = dZ3.T @ A2
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3) * (1.0 - A2 * A2)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (1.0 - A1 * A1)
    gW1 = dZ1.T @ Xp
    gb1 = dZ1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])


def loss(params, X, T):
    """Mean over the batch of the squared output error: (1/B) sum_b sum_o (Y_bo - T_bo)^2."""
    Y = forward(params, X)
    return float(np.sum((Y - T) ** 2) / Y.shape[0])


def loss_grad(params, X, T):
    """(loss, gradient) with dY = 2 (Y - T)/B."""
    Y, acts = forward(params, X, keep=True)
    B = Y.shape[0]
    return float(np.sum((Y - T) ** 2) / B), backward(params, acts, 2.0 * (Y - T) / B)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015), step counted from 1: returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def correction(params, out_scale, P, x, kappa):
    """The network's dT for one triple: h (S_re y0 + i S_im y1) / (4 pi r0^KPOW)."""
    f, h, r0, kh = features(P, x, kappa)
    y = forward(params, f)[0]
    t = out_scale[0] * y[0] + 1j * out_scale[1] * y[1]
    return h * t / (4.0 * np.pi * r0 ** KPOW)


def target(P, x, kappa, dT):
    """The scaled correction t (complex) of a triple whose correction is dT (the inverse of the
    output map above)."""
    f, h, r0, kh = features(P, x, kappa)
    return 4.0 * np.pi * r0 ** KPOW * (dT / h)
