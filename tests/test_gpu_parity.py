"""GPU parity of every C-ABI entry point against the oracle (FP64, normwise tolerances).

Workload "sphere-1280": unit icosphere level 3 (n = 1280), circle |z - 4| = 1.5 with
N = 32 trapezoidal nodes, m = 16 seeded complex Gaussian probes (seed 1).  Edge cases:
ragged n and m, strided probe blocks, single columns, complex and real wavenumbers.
Tolerance: ||gpu - oracle||_F / ||oracle||_F <= 1e-12 per node or weight set, and row by row
||gpu[r] - oracle[r]|| / ||oracle[r]|| <= 1e-12 for the per-node products and projections (a
single wrong row cannot hide below the block's norm).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def bem():
    import paper_1906_03938_amd as bem

    return bem


@pytest.fixture(scope="module")
def sphere3(bem, torch):
    from oracle import method as M

    xyz, tri = synth.icosphere(3)
    mesh = bem.Mesh(xyz, tri)
    op = M.Operator(xyz, tri)
    yield mesh, op, xyz, tri
    mesh.close()


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _row_rel(a, b):
    """Largest relative error of a row: max_r ||a[r] - b[r]|| / ||b[r]||."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_geometry_matches_oracle(sphere3, oracle_lib):
    mesh, op, xyz, tri = sphere3
    area, cen, qp, qw = mesh.geometry()
    ao, co, qo, wo = oracle_lib._clib.geometry(xyz, tri)
    assert np.abs(area - ao).max() <= 1e-15 * ao.max()
    assert np.abs(cen - co).max() <= 1e-15
    # the two implementations may list the rule's points in different orders: match each
    # point to the nearest point of the same triangle and compare weights pairwise
    d = np.linalg.norm(qp[:, :, None, :] - qo[:, None, :, :], axis=-1)  # n x 7 x 7
    nearest = d.argmin(axis=2)
    assert d.min(axis=2).max() <= 1e-15
    assert all(len(set(row)) == 7 for row in nearest)
    wmatch = np.take_along_axis(wo, nearest, axis=1)
    assert np.abs(qw - wmatch).max() <= 1e-15 * wo.max()


@pytest.mark.parametrize("kappa", [4.0, 5.5 - 1.5j, 2.5 + 1.0j, 0.0])
def test_self_terms_match_oracle(sphere3, oracle_lib, kappa):
    mesh, op, xyz, tri = sphere3
    S = mesh.self_terms([kappa]).cpu().numpy()[0]
    So = oracle_lib._clib.self_terms(xyz, tri, [kappa])[0]
    assert np.abs(S - So).max() <= 1e-14 * np.abs(So).max()


def test_assemble_apply_matches_oracle(sphere3, torch, bem):
    mesh, op, _, _ = sphere3
    V = synth.probe_block(op.n, 16, seed=1)
    kappas = [4.0, 5.5 - 1.5j, 2.5 + 1.0j, 3.14159]
    Y = mesh.assemble_apply(kappas, _dev(torch, V)).cpu().numpy()
    for k, Yk in zip(kappas, Y):
        Yo = op.apply(k, V)
        assert _rel(Yk, Yo) <= TOL, k
        assert _row_rel(Yk, Yo) <= TOL, (k, _row_rel(Yk, Yo))


@pytest.mark.parametrize("form", ["direct", "expand", "auto"])
def test_contour_moments_match_oracle(sphere3, torch, bem, form):
    from oracle import method as M

    mesh, op, _, _ = sphere3
    V = synth.probe_block(op.n, 16, seed=1)
    s, w = M.circle_nodes(4.0, 1.5, 32)
    W = M.moment_weights(s, w, 4.0, 3)
    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND, "auto": bem.FORM_AUTO}[form]
    Mg = mesh.contour_moments(s, W, _dev(torch, V), form=f).cpu().numpy()
    Mo = M.contour_moments(op, s, W, V)
    for p in range(3):
        assert _rel(Mg[p], Mo[p]) <= TOL, (form, p, _rel(Mg[p], Mo[p]))
    used, ops = mesh.last_form()
    if form == "direct":
        assert used == bem.FORM_DIRECT and ops == 32
    if form == "expand":
        assert used == bem.FORM_EXPAND and ops < 96


@pytest.mark.parametrize("form", ["direct", "expand"])
def test_rr_project_matches_oracle(sphere3, torch, bem, form):
    from oracle import method as M

    mesh, op, _, _ = sphere3
    U, _ = np.linalg.qr(synth.probe_block(op.n, 16, seed=1))
    U = np.ascontiguousarray(U)
    s, w = M.circle_nodes(4.0, 1.5, 32)
    W = M.moment_weights(s, w, 4.0, 2)
    f = bem.FORM_DIRECT if form == "direct" else bem.FORM_EXPAND
    P, Mg = mesh.rr_project(s, _dev(torch, U), W=W, form=f)
    P = P.cpu().numpy()
    Po = M.rr_project(op, s, U)
    for j in range(32):
        assert _rel(P[j], Po[j]) <= TOL, (form, j, _rel(P[j], Po[j]))
        assert _row_rel(P[j], Po[j]) <= TOL, (form, j, _row_rel(P[j], Po[j]))
    Mo = M.contour_moments(op, s, W, U)
    Mg = Mg.cpu().numpy()
    for p in range(2):
        assert _rel(Mg[p], Mo[p]) <= TOL
        assert _row_rel(Mg[p], Mo[p]) <= TOL, (form, p, _row_rel(Mg[p], Mo[p]))


@pytest.mark.parametrize("case", ["shuffled", "off_axis", "n_not_multiple_of_4", "two_circles"])
def test_direct_node_arrangements(sphere3, torch, bem, case):
    """The per-node form on node sets with and without quadruples {x +- iy, x' +- iy} (whose
    members share transcendentals in the sweep): a circle centred on the real axis in a
    shuffled order (quadruples found in any order), a circle off the axis (no conjugate
    pairs), a circle of 30 nodes (pairs but not whole quadruples) and two concentric circles
    (quadruples of both, interleaved)."""
    from oracle import method as M

    mesh, op, _, _ = sphere3
    U, _ = np.linalg.qr(synth.probe_block(op.n, 16, seed=9))
    U = np.ascontiguousarray(U)
    rng = np.random.Generator(np.random.PCG64(9))
    if case == "shuffled":
        s, w = M.circle_nodes(4.0, 1.5, 32)
        perm = rng.permutation(32)
        s, w = s[perm], w[perm]
    elif case == "off_axis":
        s, w = M.circle_nodes(4.0 + 0.25j, 1.5, 32)
    elif case == "n_not_multiple_of_4":
        s, w = M.circle_nodes(4.0, 1.5, 30)
    else:
        s1, w1 = M.circle_nodes(4.0, 1.5, 16)
        s2, w2 = M.circle_nodes(4.0, 0.75, 8)
        s, w = np.concatenate([s1, s2]), np.concatenate([w1, w2])
    W = np.ascontiguousarray(np.stack([w / (s - 4.0), w / (s - 4.0) ** 2], axis=1))
    P, Mg = mesh.rr_project(s, _dev(torch, U), W=W, form=bem.FORM_DIRECT)
    assert mesh.last_form() == (bem.FORM_DIRECT, len(s))
    P = P.cpu().numpy()
    Po = M.rr_project(op, s, U)
    for j in range(len(s)):
        assert _rel(P[j], Po[j]) <= TOL, (case, j, _rel(P[j], Po[j]))
        assert _row_rel(P[j], Po[j]) <= TOL, (case, j)
    Mo = M.contour_moments(op, s, W, U)
    Mg = Mg.cpu().numpy()
    for p in range(2):
        assert _rel(Mg[p], Mo[p]) <= TOL and _row_rel(Mg[p], Mo[p]) <= TOL, (case, p)


@pytest.mark.parametrize("form", ["direct", "expand", "cheb"])
def test_real_nodes_match_oracle(sphere3, torch, bem, form):
    """The calls the interval driver makes: projections and weighted sums on the real
    Chebyshev nodes of [2.5, 5] (the expansion then has no decay factor)."""
    from oracle import method as M

    mesh, op, _, _ = sphere3
    U, _ = np.linalg.qr(synth.probe_block(op.n, 16, seed=5))
    U = np.ascontiguousarray(U)
    kappa, coef = M.cheb_nodes(2.5, 5.0, 32)
    W = np.ascontiguousarray(coef[:3].T.astype(np.complex128))
    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND, "cheb": bem.FORM_CHEB}[form]
    P, Mg = mesh.rr_project(kappa, _dev(torch, U), W=W, form=f)
    assert mesh.last_form()[0] == f
    P = P.cpu().numpy()
    Po = M.rr_project(op, kappa, U)
    for j in range(32):
        assert _rel(P[j], Po[j]) <= TOL, (form, j, _rel(P[j], Po[j]))
    Mo = M.contour_moments(op, kappa, W, U)
    Mg = Mg.cpu().numpy()
    for p in range(3):
        assert _rel(Mg[p], Mo[p]) <= TOL, (form, p, _rel(Mg[p], Mo[p]))


@pytest.mark.parametrize("form", ["direct", "expand", "cheb"])
def test_cheb_moments_match_oracle(sphere3, torch, bem, form):
    from oracle import method as M

    mesh, op, _, _ = sphere3
    V = synth.probe_block(op.n, 16, seed=3)
    a, b, N, L = 2.5, 5.5, 24, 20
    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND, "cheb": bem.FORM_CHEB}[form]
    C = mesh.cheb_moments(a, b, N, L, _dev(torch, V), form=f).cpu().numpy()
    assert mesh.last_form()[0] == f
    Co = M.cheb_moments(op, a, b, N, L, V)
    # blocks decay with l: compare each against the scale of the leading block
    scale = np.linalg.norm(Co[0])
    for l in range(L):
        assert np.linalg.norm(C[l] - Co[l]) <= TOL * scale, (form, l)


@pytest.mark.parametrize("n_keep,m", [(1000, 5), (200, 1), (777, 33), (1280, 70)])
def test_ragged_sizes(torch, bem, oracle_lib, n_keep, m):
    """Open surfaces with n not a multiple of the 64-row tile, m not a multiple of 16,
    several column groups (m = 70), and a strided probe block."""
    xyz, tri = synth.perturbed_icosphere(3, 0.1, seed=5)
    tri = tri[:n_keep]
    from oracle import method as M

    op = M.Operator(xyz, tri)
    V = synth.probe_block(n_keep, m, seed=7)
    big = np.zeros((n_keep, m + 3), dtype=np.complex128)
    big[:, :m] = V
    Vd = _dev(torch, big)[:, :m]
    with bem.Mesh(xyz, tri) as mesh:
        for k in (3.3 - 0.4j, 6.0):
            Y = mesh.assemble_apply([k], Vd).cpu().numpy()[0]
            assert _rel(Y, op.apply(k, V)) <= TOL
        s, w = M.circle_nodes(4.0, 1.0, 12)
        W = M.moment_weights(s, w, 4.0, 2)
        Mg = mesh.contour_moments(s, W, Vd, form=bem.FORM_DIRECT).cpu().numpy()
        Mo = M.contour_moments(op, s, W, V)
        assert max(_rel(Mg[p], Mo[p]) for p in range(2)) <= TOL


def test_error_paths(torch, bem):
    from paper_1906_03938_amd import _lib

    xyz, tri = synth.icosphere(1)
    with bem.Mesh(xyz, tri) as mesh:
        V = torch.zeros((80, 4), dtype=torch.complex128, device="cuda")
        with pytest.raises(bem.BemError) as e:
            mesh.assemble_apply([4.0], V, form=0x40)
        assert e.value.status == _lib.BEM_EUNSUPPORTED
        with pytest.raises(bem.BemError) as e:
            mesh.assemble_apply([float("nan")], V)
        assert e.value.status == _lib.BEM_EINVAL
        with pytest.raises(bem.BemError) as e:
            mesh.assemble_apply([4.0 + 800j], V)
        assert e.value.status == _lib.BEM_EINVAL
        with pytest.raises(bem.BemError) as e:
            mesh.cheb_moments(2.0, 8.0, 8, 9, V)
        assert e.value.status == _lib.BEM_EINVAL
        # the Chebyshev form needs real nodes; assemble_apply takes no expansion form
        z, _, W = bem.contour_nodes(4.0, 1.0, 8, P=1)
        with pytest.raises(bem.BemError) as e:
            mesh.contour_moments(z, W, V, form=bem.FORM_CHEB)
        assert e.value.status == _lib.BEM_EUNSUPPORTED
        with pytest.raises(bem.BemError) as e:
            mesh.assemble_apply([4.0], V, form=bem.FORM_CHEB)
        assert e.value.status == _lib.BEM_EUNSUPPORTED
        # a host pointer passed as the probe block is rejected, nothing is launched
        import ctypes

        h = np.zeros((80, 4), dtype=np.complex128)
        k = np.array([4.0, 0.0])
        Y = torch.zeros((1, 80, 4), dtype=torch.complex128, device="cuda")
        st = _lib.lib().bem_assemble_apply(mesh._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1,
                                           ctypes.c_void_p(h.ctypes.data), 4, 4, ctypes.c_void_p(Y.data_ptr()), 4, 0,
                                           None)
        assert st == _lib.BEM_EINVAL
        # caller-supplied outputs are checked before anything is launched
        with pytest.raises(TypeError):
            mesh.assemble_apply([4.0], V, out=torch.zeros((1, 80, 4), dtype=torch.complex64, device="cuda"))
        with pytest.raises(ValueError):
            mesh.contour_moments(z, W, V, out=torch.zeros((1, 79, 4), dtype=torch.complex128, device="cuda"))
        with pytest.raises(ValueError):
            mesh.rr_project(z, V, out=torch.zeros((7, 4, 4), dtype=torch.complex128, device="cuda"))
        with pytest.raises(TypeError):
            mesh.assemble_sum(z, W[:, 0], out=torch.zeros((80, 80), dtype=torch.complex128))
    bad = np.array([[0, 1, 2], [0, 0, 1]], dtype=np.int32)
    with pytest.raises(bem.BemError) as e:
        bem.Mesh(xyz, bad)
    assert e.value.status == _lib.BEM_EMESH
    bem.stream_status()


def test_bitwise_deterministic(sphere3, torch, bem):
    from oracle import method as M

    mesh, op, _, _ = sphere3
    U = _dev(torch, synth.probe_block(op.n, 16, seed=2))
    s, w = M.circle_nodes(4.0, 1.5, 32)
    W = M.moment_weights(s, w, 4.0, 2)
    P1, M1 = mesh.rr_project(s, U, W=W)
    P2, M2 = mesh.rr_project(s, U, W=W)
    assert torch.equal(P1, P2) and torch.equal(M1, M2)


@pytest.mark.parametrize("form", ["direct", "expand"])
@pytest.mark.parametrize("P,m", [(1, 5), (2, 33), (2, 70), (3, 17), (3, 70), (4, 5), (4, 33), (5, 20)])
def test_folded_moments_match_unfolded(bem, torch, sphere3, form, P, m):
    """contour_moments folds up to four weight sets into the sweep (every operator of an
    entry generated, only the folds contracted; fold widths 1, 2 and 4, the last padded with
    a zero coefficient column for P = 3) and takes the unfolded route beyond (P = 5), as do
    rr_project's fused moments (every operator contracted, then recombined).  Both evaluate
    the same sums in FP64: they agree to rounding, and the result matches the oracle."""
    from oracle import method as M

    mesh, op, xyz, tri = sphere3
    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND}[form]
    z, w, W = bem.contour_nodes(4.0, 1.5, 24, P=P)
    Vm = synth.probe_block(op.n, m, seed=30 + m)
    Vmd = torch.from_numpy(Vm).to("cuda")
    Mf = mesh.contour_moments(z, W, Vmd, form=f).cpu().numpy()
    _, Mu = mesh.rr_project(z, Vmd, W=W, form=f)
    Mu = Mu.cpu().numpy()
    zo, wo = M.circle_nodes(4.0, 1.5, 24)
    Mo = M.contour_moments(op, zo, M.moment_weights(zo, wo, 4.0, P), Vm)
    for p in range(P):
        d = np.linalg.norm(Mf[p] - Mu[p]) / np.linalg.norm(Mu[p])
        e = np.linalg.norm(Mf[p] - Mo[p]) / np.linalg.norm(Mo[p])
        print(form, P, m, p, "folded vs unfolded", d, "vs oracle", e, flush=True)
        assert d <= 1e-13 and e <= TOL


def test_taylor_plan_stops_at_the_reach_of_the_weights(bem, torch, sphere3):
    """Moment weights of a circle about the expansion centre reach one Taylor operator each
    (the trapezoidal rule integrates t^k exactly), so the plan for moments of orders 1-3 stops
    at the length unit of 8 operators and the moments still match the oracle's per-node sums;
    resolvent weights w_j / (lam - z_j) reach further (a longer plan, still within rr_project's
    full length), also matching the oracle."""
    from oracle import method as M

    mesh, op, _, _ = sphere3
    V = synth.probe_block(op.n, 8, seed=4)
    Vd = _dev(torch, V)
    z, w, W = bem.contour_nodes(4.0, 1.5, 32, P=3)
    s, wo = M.circle_nodes(4.0, 1.5, 32)
    Mg = mesh.contour_moments(z, W, Vd, form=bem.FORM_EXPAND).cpu().numpy()
    assert mesh.last_form() == (bem.FORM_EXPAND, 8)
    Mo = M.contour_moments(op, s, M.moment_weights(s, wo, 4.0, 3), V)
    for p in range(3):
        assert _rel(Mg[p], Mo[p]) <= TOL, (p, _rel(Mg[p], Mo[p]))
    mesh.rr_project(z, Vd, form=bem.FORM_EXPAND)
    L_full = mesh.last_form()[1]
    lam = 5.3
    Wr = np.ascontiguousarray((w / (lam - z))[:, None])
    Mr = mesh.contour_moments(z, Wr, Vd, form=bem.FORM_EXPAND).cpu().numpy()
    reach = mesh.last_form()[1]
    print("full length", L_full, "resolvent reach", reach, flush=True)
    assert 8 < reach <= L_full
    Mro = M.contour_moments(op, s, (wo / (lam - s))[:, None], V)
    assert _rel(Mr[0], Mro[0]) <= TOL, _rel(Mr[0], Mro[0])
