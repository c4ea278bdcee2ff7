"""GPU checks of the learned near-field correction against the oracle (oracle/nfnet.py,
oracle/bem_oracle.c), through the C ABI.

* labels (bem_nf_labels): integral minus 7-point value against the oracle's adaptive cubature
  minus its own 7-point sum, 1e-12 of the integral;
* inputs (bem_net_features): the FP32 inputs and FP64 frame quantities against the oracle's map
  on triples in general position (rotated, translated, scaled);
* forward pass and gradient (bem_net_forward, bem_net_gradient, FP32 on the matrix cores)
  against the oracle's FP64 network and back-propagation: 1e-5 and 1e-4 relative;
* one Adam step against the oracle's;
* training on the GPU: the loss falls, the validation errors are finite, trust flags follow
  the bound;
* the learned moments (bem_nearfield_moments_net): with no bin trusted they equal the
  quadrature's bitwise; trusted, each pair's FP16 correction matches the oracle's FP64
  network on the same parameters to 1e-2 of the largest correction, and the corrected moments
  beat the uncorrected ones against the quadrature reference;
* the gain on the near-field workload "harmonic-499280" (geodesic f = 158 sphere with
  harmonic bumps, eta = 2, |z - 5| = 1.5, N = 32, P = 2, m = 64): error of the network's
  correction against the quadrature's, and both times.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1906_03938_amd as bem
    from oracle import _clib
    from oracle import nfnet as O
    from paper_1906_03938_amd import _lib, nfnet

    assert torch.cuda.is_available()
    return bem, _lib, nfnet, O, _clib, torch


def _triples(n, seed, scale=True):
    """Canonical samples moved by seeded rigid motions and scalings."""
    P, x, kh = synth.nearfield_samples(n, seed)
    if not scale:
        return P, x, kh
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    Ps, xs, ks = [], [], []
    for i in range(n):
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        s = rng.uniform(0.01, 3.0)
        t = rng.standard_normal(3)
        Ps.append(s * P[i] @ q.T + t)
        xs.append(s * q @ x[i] + t)
        ks.append(kh[i] / s)
    return np.array(Ps), np.array(xs), np.array(ks)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_labels_match_oracle(env):
    bem, _lib, nfnet, O, _clib, torch = env
    P, x, k = _triples(48, 21)
    dT = _lib.nf_labels(_dev(torch, P.reshape(-1, 9)), _dev(torch, x), _dev(torch, k)).cpu().numpy()
    bary, w = _clib.radon7()
    for s in range(len(k)):
        I = _clib.tri_integral(x[s], P[s], [k[s]])[0]
        A = 0.5 * np.linalg.norm(np.cross(P[s, 1] - P[s, 0], P[s, 2] - P[s, 0]))
        r = np.linalg.norm(x[s][None] - bary @ P[s], axis=1)
        seven = np.sum(A * w * np.exp(1j * k[s] * r) / (4 * np.pi * r))
        assert abs(dT[s] - (I - seven)) <= 1e-12 * abs(I), (s, dT[s], I - seven)


def test_features_match_oracle(env):
    bem, _lib, nfnet, O, _clib, torch = env
    P, x, k = _triples(64, 22)
    X, aux = _lib.net_features(_dev(torch, P.reshape(-1, 9)), _dev(torch, x), _dev(torch, k))
    X, aux = X.cpu().numpy(), aux.cpu().numpy()
    for s in range(len(k)):
        f, h, r0, kh = O.features(P[s], x[s], k[s])
        assert np.allclose(X[s, :O.F], f, rtol=1e-6, atol=1e-6), s
        assert np.all(X[s, O.F:] == 0.0)
        assert abs(aux[s, 0] - h) <= 1e-13 * h and abs(aux[s, 1] - r0) <= 1e-12 * r0
        assert abs(aux[s, 2] + 1j * aux[s, 3] - kh) <= 1e-13 * abs(kh)


def _oracle_params(O, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal(O.N_PARAMS) * 0.15
    O.split(p)[0][:, O.F:] = 0.0
    return p


@pytest.mark.parametrize("B", [1, 100, 8192])
def test_forward_and_gradient_match_oracle(env, B):
    bem, _lib, nfnet, O, _clib, torch = env
    rng = np.random.Generator(np.random.PCG64(23 + B))
    p = _oracle_params(O, 24)
    X = np.zeros((B, O.F_PAD))
    X[:, :O.F] = rng.standard_normal((B, O.F))
    T = rng.standard_normal((B, 2))
    pd = _dev(torch, p.astype(np.float32))
    Xd = _dev(torch, X.astype(np.float32))
    Y = _lib.net_forward(pd, Xd).cpu().numpy()
    # the oracle on the same FP32-rounded parameters and inputs
    p32, X32 = p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64)
    Yo = O.forward(p32, X32)
    assert np.abs(Y - Yo).max() <= 1e-5 * np.abs(Yo).max()
    g, loss = _lib.net_gradient(pd, Xd, _dev(torch, T.astype(np.float32)))
    lo, go = O.loss_grad(p32, X32, T.astype(np.float32).astype(np.float64))
    g = g.cpu().numpy()
    assert abs(loss.item() - lo) <= 1e-5 * lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    for blk, gb in zip(O.split(g), O.split(go)):  # every parameter block on its own
        assert np.linalg.norm(blk - gb) <= 1e-4 * max(np.linalg.norm(gb), 1e-30 + 1e-6 * np.linalg.norm(go))


def test_adam_matches_oracle(env):
    bem, _lib, nfnet, O, _clib, torch = env
    rng = np.random.Generator(np.random.PCG64(25))
    p = rng.standard_normal(O.N_PARAMS).astype(np.float32)
    g = rng.standard_normal(O.N_PARAMS).astype(np.float32)
    m = (0.1 * rng.standard_normal(O.N_PARAMS)).astype(np.float32)
    v = (0.01 * rng.uniform(0, 1, O.N_PARAMS)).astype(np.float32)
    pd, gd, md, vd = (_dev(torch, a) for a in (p, g, m, v))
    _lib.net_adam(pd, gd, md, vd, 7, 3e-3)
    po, mo, vo = O.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64), v.astype(np.float64), 7,
                        3e-3)
    # FP32 against FP64 (beta1, beta2 are not exact in FP32: 1 - beta2 is off by 1.3e-5 relative)
    assert np.abs(pd.cpu().numpy() - po).max() <= 1e-6
    assert np.abs(md.cpu().numpy() - mo).max() <= 1e-5 * np.abs(mo).max()
    assert np.abs(vd.cpu().numpy() - vo).max() <= 1e-4 * np.abs(vo).max()


@pytest.fixture(scope="module")
def trained(env):
    bem, _lib, nfnet, O, _clib, torch = env
    t0 = time.perf_counter()
    net = nfnet.train(train_count=400_000, val_count=50_000, seed=31, steps=20000, batch=2048, bound=0.25,
                      log=lambda s: print(s, flush=True))
    print(f"training {time.perf_counter() - t0:.1f} s; per-bin validation error {np.round(net.bin_error, 4)}; "
          f"share of all {np.round(net.bin_share, 4)}; counts {net.bin_count}; trusted {net.bin_trusted}", flush=True)
    return net


def test_training_reduces_loss(trained):
    h = trained.history
    assert h[-1][1] < 0.1 * h[0][1], h
    assert all(np.isfinite(e) for e in trained.bin_error)
    assert trained.bin_trusted == [e <= trained.bound / np.sqrt(8) for e in trained.bin_share]
    assert any(trained.bin_trusted)


def _mesh_case(bem, torch):
    xyz, tri = synth.perturbed_icosphere(3, 0.1, seed=5)
    z, w, W = bem.contour_nodes(5.0, 1.5, 16, P=2)
    return xyz, tri, z, W


def test_untrusted_model_equals_quadrature(env, trained):
    bem, _lib, nfnet, O, _clib, torch = env
    xyz, tri, z, W = _mesh_case(bem, torch)
    V = _dev(torch, synth.probe_block(len(tri), 8, seed=3))
    none = trained.with_trust([False] * 8)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Mq = mesh.nearfield_moments(z, W, V)
        Mn, fb = mesh.nearfield_moments_net(none.c_model(), z, W, V, count_fallback=True)
        pairs = mesh.nearfield_list()[1].size
    assert fb == pairs
    assert torch.equal(Mq, Mn)


def test_inference_matches_oracle_network(env, trained):
    """V = I: the learned moments with W = I are the per-pair corrections dT_ab(z_j) themselves,
    compared pair by pair (every 8th row) with the oracle's FP64 network on the same (FP32)
    parameters, for the pairs inside the trust region (with a margin at its edges)."""
    bem, _lib, nfnet, O, _clib, torch = env
    xyz, tri = synth.icosphere(3)
    n = len(tri)
    z = np.array([4.6 + 0.3j, 5.2 - 0.4j])
    W = np.eye(2, dtype=np.complex128)
    allt = trained.with_trust([True] * 8)
    params = trained.params.cpu().numpy().astype(np.float64)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Mn, fb = mesh.nearfield_moments_net(allt.c_model(), z, W, _dev(torch, np.eye(n, dtype=np.complex128)),
                                           count_fallback=True)
        rp, col = mesh.nearfield_list()
    Mn = Mn.cpu().numpy()
    P3 = xyz[tri]
    cen = P3.mean(axis=1)
    tmin = np.tan(np.deg2rad(trained.min_angle_deg))
    kre, kim = np.abs(z.real).max(), np.abs(z.imag).max()
    got, ref = [], []
    for a in range(0, n, 8):
        for i in range(rp[a], rp[a + 1]):
            b = col[i]
            p, q, u, v, w, h = O.canonical(P3[b], cen[a])
            d = nfnet.unit_distance(np.array([p]), np.array([q]), np.array([u]), np.array([v]), np.array([w]))[0]
            m = 1e-9
            if not (d >= trained.dmin + m and q >= (1 - p) * tmin + m and q >= p * tmin + m
                    and kre * h <= trained.kh_re_max - m and kim * h <= trained.kh_im_max - m):
                continue  # outside the trust region (or at its edge): quadrature
            for j in range(2):
                got.append(Mn[j, a, b])
                ref.append(O.correction(params, trained.out_scale, P3[b], cen[a], z[j]))
    got, ref = np.array(got), np.array(ref)
    print(f"{got.size} pair-node corrections, fallback pairs {fb}; max |fp16 - oracle| / max |dT| = "
          f"{np.abs(got - ref).max() / np.abs(ref).max():.2e}", flush=True)
    assert got.size > 100
    assert np.abs(got - ref).max() <= 1e-2 * np.abs(ref).max()


def test_frozen_inference_matches_oracle_network(env, trained):
    """Frozen wavenumber (bem_net_model.freeze_tol > 0): one evaluation per pair at the centre
    kc of the nodes' bounding box, used for every node.  With W = I and V = I the moments are
    the per-pair corrections: both nodes get the same value, equal to the oracle's FP64 network
    at kc for the pairs inside the trust region; with a bound no pair meets (1e-12) every pair
    takes the quadrature and the moments equal the quadrature's bitwise."""
    bem, _lib, nfnet, O, _clib, torch = env
    xyz, tri = synth.icosphere(3)
    n = len(tri)
    z = np.array([4.6 + 0.3j, 5.2 - 0.4j])
    kc = complex(0.5 * (z.real.min() + z.real.max()), 0.5 * (z.imag.min() + z.imag.max()))
    W = np.eye(2, dtype=np.complex128)
    allt = trained.with_trust([True] * 8)
    params = trained.params.cpu().numpy().astype(np.float64)
    I = _dev(torch, np.eye(n, dtype=np.complex128))
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Mf, fb = mesh.nearfield_moments_net(allt.frozen(1e9).c_model(), z, W, I, count_fallback=True)
        Mz, fbz = mesh.nearfield_moments_net(allt.frozen(1e-12).c_model(), z, W, I, count_fallback=True)
        Mq = mesh.nearfield_moments(z, W, I)
        rp, col = mesh.nearfield_list()
    assert fbz == col.size and torch.equal(Mz, Mq)
    Mf = Mf.cpu().numpy()
    P3 = xyz[tri]
    cen = P3.mean(axis=1)
    tmin = np.tan(np.deg2rad(trained.min_angle_deg))
    kre, kim = np.abs(z.real).max(), np.abs(z.imag).max()
    got, ref = [], []
    for a in range(0, n, 8):
        for i in range(rp[a], rp[a + 1]):
            b = col[i]
            p, q, u, v, w, h = O.canonical(P3[b], cen[a])
            d = nfnet.unit_distance(np.array([p]), np.array([q]), np.array([u]), np.array([v]), np.array([w]))[0]
            m = 1e-9
            if not (d >= trained.dmin + m and q >= (1 - p) * tmin + m and q >= p * tmin + m
                    and kre * h <= trained.kh_re_max - m and kim * h <= trained.kh_im_max - m):
                continue
            assert Mf[0, a, b] == Mf[1, a, b]
            got.append(Mf[0, a, b])
            ref.append(O.correction(params, trained.out_scale, P3[b], cen[a], kc))
    got, ref = np.array(got), np.array(ref)
    print(f"{got.size} frozen pair corrections, fallback pairs {fb}; max |fp16 - oracle| / max |dT| = "
          f"{np.abs(got - ref).max() / np.abs(ref).max():.2e}", flush=True)
    assert got.size > 50
    assert np.abs(got - ref).max() <= 1e-2 * np.abs(ref).max()


def test_learned_correction_beats_no_correction(env, trained):
    """Moments of the corrected operator (7-point sweep plus near-field correction) against the
    quadrature reference: with the network's correction the error is a fraction of the correction
    itself, the error of leaving it out, for the leading moment; the derivative moment is
    reported (per-node FP16 rounding does not cancel in its weights)."""
    bem, _lib, nfnet, O, _clib, torch = env
    xyz, tri, z, W = _mesh_case(bem, torch)
    V = _dev(torch, synth.probe_block(len(tri), 8, seed=3))
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        M7 = mesh.contour_moments(z, W, V).cpu().numpy()
        Dq = mesh.nearfield_moments(z, W, V).cpu().numpy()
        Dn, fb = mesh.nearfield_moments_net(trained.c_model(), z, W, V, count_fallback=True)
        Dn = Dn.cpu().numpy()
        pairs = mesh.nearfield_list()[1].size
    assert fb < pairs
    gains = []
    for p in range(2):
        ref = np.linalg.norm(M7[p] + Dq[p])
        e_net = np.linalg.norm(Dn[p] - Dq[p]) / ref
        e_none = np.linalg.norm(Dq[p]) / ref
        gains.append(e_none / e_net)
        print(f"moment {p + 1}: corrected-moment error with the network {e_net:.3e}, without a correction "
              f"{e_none:.3e} (gain {e_none / e_net:.1f}); fallback {fb}/{pairs}", flush=True)
    assert gains[0] >= 5.0


def test_gain_on_eigenvalues(env, trained):
    """sphere-1280 (|z - 4| < 1.5, N = 32, 16 probes): eigenvalues of the corrected operator with
    the network's correction against the oracle's (quadrature) corrected eigenvalues; the error
    is at most a tenth of the shift the correction makes (the error of leaving it out)."""
    import os

    bem, _lib, nfnet, O, _clib, torch = env
    from paper_1906_03938_amd.eig import eigs_in_contour

    g = os.path.join(os.path.dirname(__file__), "golden")
    ref_nf = np.loadtxt(os.path.join(g, "sphere1280_nearfield_eigs.txt"))
    ref = np.loadtxt(os.path.join(g, "sphere1280_eigs.txt"))
    lam_nf = np.sort_complex(ref_nf[:, 0] + 1j * ref_nf[:, 1])
    lam_plain = np.sort_complex(ref[:, 0] + 1j * ref[:, 1])
    xyz, tri = synth.icosphere(3)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        # the network's corrections carry FP16 rounding (~1e-3 of each correction, ~1e-6 of the
        # operator): residuals stop near that level
        lam, X, res, outer = eigs_in_contour(mesh, 4.0, 1.5, 32, synth.probe_block(1280, 16, seed=1), tol=1e-5,
                                             max_outer=6, nearfield=trained)
    lam = np.sort_complex(lam)
    assert lam.size == lam_nf.size and res.max() <= 1e-5
    e_net = np.abs(lam - lam_nf).max() / np.abs(lam_nf).max()
    e_none = np.abs(lam_plain - lam_nf).max() / np.abs(lam_nf).max()
    print(f"eigenvalues: network-corrected error {e_net:.3e}, uncorrected {e_none:.3e} (gain {e_none / e_net:.1f}); "
          f"{outer} outer iterations, max residual {res.max():.1e}", flush=True)
    assert e_net <= 0.1 * e_none


def test_gain_on_harmonic_sphere(env, trained):
    """Config 5's mesh and contour (harmonic-499280, |z - 5| = 1.5, N = 32, P = 2, m = 64): the
    network's correction of the leading moment within half of the quadrature's, per node and
    frozen at the contour centre (freeze_tol 1e-2), each trusting some pairs; the frozen mode
    (one evaluation per pair) faster than the per-node quadrature, and the quadrature's series
    form (exact to rounding, also one pass over the pairs) faster than the per-node quadrature.
    Times are printed."""
    bem, _lib, nfnet, O, _clib, torch = env
    xyz, tri = synth.harmonic_sphere(158, seed=5)
    n = len(tri)
    z, w, W = bem.contour_nodes(5.0, 1.5, 32, P=2)
    V = _dev(torch, synth.probe_block(n, 64, seed=5))
    frozen = trained.frozen(1e-2)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        pairs = mesh.nearfield_list()[1].size
        Mq = mesh.nearfield_moments(z, W, V)
        Mn, fb = mesh.nearfield_moments_net(trained.c_model(), z, W, V, count_fallback=True)
        Mf, fbf = mesh.nearfield_moments_net(frozen.c_model(), z, W, V, count_fallback=True)
        torch.cuda.synchronize()
        times = {}
        def per_node():
            mesh.set_nearfield_mode(bem.NF_NODES)
            mesh.nearfield_moments(z, W, V, out=Mq.zero_())
            mesh.set_nearfield_mode(bem.NF_AUTO)

        for name, f in (("quadrature", lambda: mesh.nearfield_moments(z, W, V, out=Mq.zero_())),
                        ("per-node quadrature", per_node),
                        ("network", lambda: mesh.nearfield_moments_net(trained.c_model(), z, W, V, out=Mn.zero_())),
                        ("frozen", lambda: mesh.nearfield_moments_net(frozen.c_model(), z, W, V, out=Mf.zero_()))):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            times[name] = e0.elapsed_time(e1)
        err = [float(torch.linalg.vector_norm(Mn[p] - Mq[p]) / torch.linalg.vector_norm(Mq[p])) for p in range(2)]
        errf = [float(torch.linalg.vector_norm(Mf[p] - Mq[p]) / torch.linalg.vector_norm(Mq[p])) for p in range(2)]
    print(f"harmonic-499280: {pairs} pairs, fallback {fb} (frozen {fbf}); correction rel err per node {err}, "
          f"frozen {errf}; quadrature (series form) {times['quadrature']:.1f} ms, per-node quadrature "
          f"{times['per-node quadrature']:.1f} ms, network {times['network']:.1f} ms, "
          f"frozen {times['frozen']:.1f} ms", flush=True)
    assert err[0] <= 0.5 and errf[0] <= 0.5
    assert fb < pairs and fbf < pairs
    assert times["frozen"] < times["per-node quadrature"]
    assert times["quadrature"] < times["per-node quadrature"]
