"""Training driver of the learned near-field correction.

The network (include/bemrat.h, "learned near-field correction") is trained on the GPU by the
library's own kernels: seeded (triangle, target, wavenumber) triples in the unit frame of the
source triangle (synth.nearfield_samples) are labelled by the library's polar quadrature
(bem_nf_labels), turned into inputs (bem_net_features), and fitted by mini-batch Adam on the
mean squared error of the scaled correction (bem_net_gradient, bem_net_adam).  A held-out set
labelled the same way gives the validation error per distance bin; bins whose error exceeds
the bound are left to the quadrature (the model's trust region), which stays the reference.

Host work here is data movement and bookkeeping only: the sampling of inputs, the output scale
(a standard deviation of the labels), the learning-rate schedule and the per-bin error
statistics of the validation predictions.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib

KPOW = 4                   # the scaled target is 4 pi r0^KPOW dT / h
BIN_EDGES = [0.15, 0.2, 0.3, 0.45, 0.65, 0.9, 1.2, 1.6, 1e9]
DMIN = 0.15                # nearest trusted target-triangle distance (units of h)
MIN_ANGLE = 20.0           # smallest trusted triangle angle (degrees)
KH_RE = (0.0, 1.0)         # trained range of Re(kappa h)
KH_IM = (-0.3, 0.3)        # trained range of Im(kappa h)


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights (bound sqrt(6/(fan_in + fan_out))), zero biases; W1's unused input
    columns 19..31 zero.  Seeded by numpy PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, F, FP, O = 128, 19, 32, 2
    parts = []
    W1 = np.zeros((H, FP))
    W1[:, :F] = rng.uniform(-1, 1, (H, F)) * np.sqrt(6.0 / (F + H))
    parts += [W1, np.zeros(H)]
    for _ in range(2):
        parts += [rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / (2 * H)), np.zeros(H)]
    parts += [rng.uniform(-1, 1, (O, H)) * np.sqrt(6.0 / (H + O)), np.zeros(O)]
    p = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert p.size == _lib.NET_PARAMS
    return p


def unit_distance(p, q, u, v, w):
    """Distance of unit-frame targets (u, v, w) to the triangles (0,0), (1,0), (p,q) (arrays)."""
    def seg(ax, ay, bx, by):
        dx, dy = bx - ax, by - ay
        t = np.clip(((u - ax) * dx + (v - ay) * dy) / (dx * dx + dy * dy), 0.0, 1.0)
        return np.sqrt((u - ax - t * dx) ** 2 + (v - ay - t * dy) ** 2 + w * w)

    d11 = p * p + q * q
    den = d11 - p * p
    lb = (d11 * u - p * (u * p + v * q)) / den
    lc = ((u * p + v * q) - p * u) / den
    inside = (lb >= 0) & (lc >= 0) & (lb + lc <= 1)
    out = np.minimum(np.minimum(seg(0.0, 0.0, 1.0, 0.0), seg(1.0, 0.0, p, q)), seg(p, q, 0.0, 0.0))
    return np.where(inside, np.abs(w), out)


@dataclass
class NearFieldNet:
    """A trained network, its output scales and its trust region."""
    params: object                     # torch float32 CUDA tensor, NET_PARAMS
    out_scale: tuple
    bin_edges: list = field(default_factory=lambda: list(BIN_EDGES))
    bin_error: list = field(default_factory=list)    # validation error within each bin (relative)
    bin_share: list = field(default_factory=list)    # each bin's error relative to all corrections
    bin_count: list = field(default_factory=list)
    bin_trusted: list = field(default_factory=list)
    bound: float = 0.2
    dmin: float = DMIN
    min_angle_deg: float = MIN_ANGLE
    kh_re_max: float = KH_RE[1]
    kh_im_max: float = KH_IM[1]
    freeze_tol: float = 0.0                          # > 0: one evaluation per pair (bem_net_model)
    history: list = field(default_factory=list)      # (step, loss)
    stats: dict = field(default_factory=dict)

    def c_model(self):
        """The bem_net_model struct of this network (keeps a reference to the parameters)."""
        m = _lib.NetModelC()
        m.params = ctypes.c_void_p(self.params.data_ptr())
        m.out_scale[0], m.out_scale[1] = float(self.out_scale[0]), float(self.out_scale[1])
        m.dmin = self.dmin
        m.min_angle_deg = self.min_angle_deg
        m.kh_re_max = self.kh_re_max
        m.kh_im_max = self.kh_im_max
        for i, e in enumerate(self.bin_edges):
            m.bin_edges[i] = e
        for i, t in enumerate(self.bin_trusted):
            m.bin_trusted[i] = 1 if t else 0
        m.freeze_tol = float(self.freeze_tol)
        self._c = m
        return m

    def with_trust(self, trusted):
        """A copy whose bins are trusted as given (a list of 8 booleans)."""
        c = NearFieldNet(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        c.bin_trusted = [bool(t) for t in trusted]
        return c

    def frozen(self, tol=1e-2):
        """A copy evaluated once per pair at the centre of the node set, for the pairs whose
        estimated relative change of the correction over the nodes (spread x |kappa|max x h^2)
        is at most tol (bem_net_model.freeze_tol); 0 restores per-node evaluation."""
        c = NearFieldNet(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        c.freeze_tol = float(tol)
        return c


def _dataset(count, seed, torch):
    """Samples, labels and inputs on the device: (X, aux, dT, P, x)."""
    import synth

    P, x, kh = synth.nearfield_samples(count, seed, dmin=DMIN, kh_re=KH_RE, kh_im=KH_IM, min_angle_deg=MIN_ANGLE)
    Pd = torch.from_numpy(np.ascontiguousarray(P.reshape(count, 9))).to("cuda")
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    kd = torch.from_numpy(np.ascontiguousarray(kh)).to("cuda")  # h = 1: kappa = kappa h
    dT = _lib.nf_labels(Pd, xd, kd)
    X, aux = _lib.net_features(Pd, xd, kd)
    return X, aux, dT, P, x


def _targets(aux, dT):
    """The scaled correction t = 4 pi r0^KPOW dT / h (complex, host)."""
    h, r0 = aux[:, 0], aux[:, 1]
    return 4.0 * np.pi * r0 ** KPOW * dT / h


def predict(net: NearFieldNet, X, aux):
    """dT from the FP32 forward pass (host arrays)."""
    Y = _lib.net_forward(net.params, X).cpu().numpy().astype(np.float64)
    a = aux.cpu().numpy() if hasattr(aux, "cpu") else aux
    h, r0 = a[:, 0], a[:, 1]
    t = net.out_scale[0] * Y[:, 0] + 1j * net.out_scale[1] * Y[:, 1]
    return h * t / (4.0 * np.pi * r0 ** KPOW)


def train(train_count: int = 2_000_000, val_count: int = 100_000, seed: int = 11, steps: int = 40000,
          batch: int = 2048, lr_max: float = 2e-3, bound: float = 0.2, log=None) -> NearFieldNet:
    """Trains the network on the GPU; returns it with its validation errors and trust region."""
    import torch

    t0 = time.perf_counter()
    X, aux, dT, _, _ = _dataset(train_count, seed, torch)
    t = _targets(aux.cpu().numpy(), dT.cpu().numpy())
    scale = (float(np.std(t.real)), float(np.std(t.imag)))
    T = torch.from_numpy(np.stack([t.real / scale[0], t.imag / scale[1]], axis=1).astype(np.float32)).to("cuda")
    Xv, auxv, dTv, Pv, xv = _dataset(val_count, seed + 1, torch)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    params = torch.from_numpy(init_params(seed)).to("cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    work = _lib.net_work(batch)
    nb = train_count // batch
    net = NearFieldNet(params=params, out_scale=scale, bound=bound)
    warm = max(1, steps // 20)
    t1 = time.perf_counter()
    for step in range(1, steps + 1):
        # one-cycle schedule: linear warm-up, then cosine decay to lr_max / 100
        if step <= warm:
            lr = lr_max * step / warm
        else:
            c = (step - warm) / max(1, steps - warm)
            lr = lr_max * (0.01 + 0.99 * 0.5 * (1.0 + np.cos(np.pi * c)))
        b0 = ((step - 1) % nb) * batch
        _lib.net_gradient(params, X[b0:b0 + batch], T[b0:b0 + batch], work=work, grad=grad, loss=loss)
        _lib.net_adam(params, grad, m, v, step, lr)
        if step == 1 or step % 5000 == 0 or step == steps:
            net.history.append((step, float(loss.item())))
            if log:
                log(f"step {step}: loss {net.history[-1][1]:.3e} ({time.perf_counter() - t1:.1f} s)")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    # validation: each distance bin's share of the error, relative to all the corrections (a
    # bin is trusted when its share stays within bound / sqrt(bins), so that the bins trusted
    # together stay within the bound); and, for reference, the error within each bin
    pred = predict(net, Xv, auxv)
    ref = dTv.cpu().numpy()
    d = unit_distance(Pv[:, 2, 0], Pv[:, 2, 1], xv[:, 0], xv[:, 1], np.abs(xv[:, 2]))
    total = float(np.sum(np.abs(ref) ** 2))
    nbins = len(BIN_EDGES) - 1
    net.bin_error, net.bin_share, net.bin_count, net.bin_trusted = [], [], [], []
    for i in range(nbins):
        sel = (d >= BIN_EDGES[i]) & (d < BIN_EDGES[i + 1])
        sq = float(np.sum(np.abs(pred[sel] - ref[sel]) ** 2))
        err = float(np.sqrt(sq / np.sum(np.abs(ref[sel]) ** 2))) if sel.any() else float("inf")
        share = float(np.sqrt(sq / total)) if sel.any() else float("inf")
        net.bin_error.append(err)
        net.bin_share.append(share)
        net.bin_count.append(int(sel.sum()))
        net.bin_trusted.append(bool(share <= bound / np.sqrt(nbins)))
    net.stats = {"train_samples": train_count, "val_samples": val_count, "steps": steps, "batch": batch,
                 "data_seconds": t_data, "train_seconds": t_train,
                 "val_rel_err": float(np.sqrt(np.sum(np.abs(pred - ref) ** 2) / np.sum(np.abs(ref) ** 2)))}
    return net
