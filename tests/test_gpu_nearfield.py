"""GPU parity of the near-field correction against the oracle's adaptive cubature.

Workloads: unit icosphere level 3 (n = 1280, 34 near pairs per row at eta = 2), the box
1.0 x 0.8 x 0.6 on a 10 x 8 x 6 grid (coplanar neighbours, collocation points on the edge
lines of other triangles), a randomly perturbed icosphere (level 3, amplitude 0.05, seed 5:
uneven triangles), circle |z - 4| = 1.5 with N = 16 trapezoidal nodes, m = 16 seeded
probes.  The near-pair list is index work and must be identical; the moments of the
corrected operator (contour_moments + bem_nearfield_moments) must agree with the oracle's
to ||gpu - oracle||_F / ||oracle||_F <= 1e-12 per weight set, and the correction alone to
1e-12 of the corrected moments (the correction is a difference of two nearly equal values,
so its own relative error is larger by the ratio of the entries to the corrections).
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


def _mesh(name):
    if name == "sphere":
        return synth.icosphere(3)
    if name == "box":
        return synth.box_surface((1.0, 0.8, 0.6), (10, 8, 6))
    return synth.perturbed_icosphere(3, 0.05, 5)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _correction_ref(xyz, tri, eta, z, W, V):
    """sum_j W[j, p] dT(z_j) V from the oracle's per-pair corrections."""
    import scipy.sparse as sp
    from oracle import _clib

    n = len(tri)
    rp, col, dT = _clib.nearfield_correction(xyz, tri, eta, z)
    rows = np.repeat(np.arange(n), np.diff(rp))
    out = np.zeros((W.shape[1], n, V.shape[1]), dtype=np.complex128)
    for j in range(len(z)):
        D = sp.csr_matrix((dT[j], (rows, col)), shape=(n, n))
        Y = D @ V
        for p in range(W.shape[1]):
            out[p] += W[j, p] * Y
    return out


@pytest.mark.parametrize("name", ["sphere", "box", "perturbed"])
def test_near_pair_list_is_identical(bem, torch, oracle_lib, name):
    from oracle import _clib

    xyz, tri = _mesh(name)
    with bem.Mesh(xyz, tri) as mesh:
        rp0, col0 = mesh.nearfield_list()
        assert col0.size == 0 and not rp0.any()
        for eta in (1.0, 2.0, 3.0):
            mesh.set_nearfield(eta)
            rp, col = mesh.nearfield_list()
            rpo, colo = _clib.near_pairs(xyz, tri, eta)
            assert np.array_equal(rp, rpo) and np.array_equal(col, colo), (name, eta)


@pytest.mark.parametrize("name", ["sphere", "box", "perturbed"])
def test_corrected_moments_match_oracle(bem, torch, oracle_lib, name):
    from oracle import method as M

    xyz, tri = _mesh(name)
    n = len(tri)
    z, w, W = bem.contour_nodes(4.0, 1.5, 16, P=2)
    V = synth.probe_block(n, 16, seed=1)
    eta = 2.0
    corr = _correction_ref(xyz, tri, eta, z, W, V)
    base = M.contour_moments(M.Operator(xyz, tri), z, W, V)
    full = base + corr
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(eta)
        Vd = _dev(torch, V)
        Mg = mesh.contour_moments(z, W, Vd)
        mesh.nearfield_moments(z, W, Vd, out=Mg)
        Cg = mesh.nearfield_moments(z, W, Vd).cpu().numpy()
        Mg = Mg.cpu().numpy()
    for p in range(W.shape[1]):
        e_full = np.linalg.norm(Mg[p] - full[p]) / np.linalg.norm(full[p])
        e_corr = np.linalg.norm(Cg[p] - corr[p]) / np.linalg.norm(full[p])
        print(f"{name} p={p}: corrected moments rel err {e_full:.2e}, correction err {e_corr:.2e} "
              f"(|corr|/|M| = {np.linalg.norm(corr[p]) / np.linalg.norm(full[p]):.1e})")
        assert e_full <= TOL and e_corr <= TOL
    # the correction is not negligible at this size: it changes the moments well above the
    # parity tolerance
    assert np.linalg.norm(corr[0]) >= 1e3 * TOL * np.linalg.norm(full[0])


@pytest.mark.parametrize("level,keep,eta,series", [(2, 301, 2.5, False), (3, 1201, 2.0, True)])
def test_many_weight_sets_ragged_and_strided(bem, torch, oracle_lib, level, keep, eta, series):
    """P = 11 (two launches of up to 8 weight sets), per-node weights (W = I gives
    dT(z_j) V), m = 5 inside a strided probe block, a ragged mesh size; on the coarse mesh the
    series would need more than 32 terms (per-node form), on the finer one it takes the series
    form."""
    xyz, tri = synth.perturbed_icosphere(level, 0.08, 7)
    tri = tri[:keep]
    used = np.unique(tri)
    remap = -np.ones(len(xyz), dtype=np.int64)
    remap[used] = np.arange(used.size)
    xyz, tri = xyz[used], remap[tri].astype(np.int32)
    n = len(tri)
    rng = np.random.default_rng(3)
    z = np.array([3.0 + 0.5j, 4.5 - 0.2j, 2.0, 5.5 + 1.0j, 4.0 + 0.0j])
    W = rng.normal(size=(5, 11)) + 1j * rng.normal(size=(5, 11))
    Vfull = synth.probe_block(n, 9, seed=2)
    V = Vfull[:, 2:7]
    corr = _correction_ref(xyz, tri, eta, z, W, V)
    corr_id = _correction_ref(xyz, tri, eta, z, np.eye(5, dtype=np.complex128), V)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(eta)
        Vd = _dev(torch, Vfull)[:, 2:7]
        Cg = mesh.nearfield_moments(z, W, Vd).cpu().numpy()
        assert (mesh.nearfield_last_terms() > 0) == series
        Ig = mesh.nearfield_moments(z, np.eye(5), Vd).cpu().numpy()
    for p in range(11):
        assert np.linalg.norm(Cg[p] - corr[p]) <= 1e-11 * np.linalg.norm(corr[p])
    for j in range(5):
        assert np.linalg.norm(Ig[j] - corr_id[j]) <= 1e-11 * np.linalg.norm(corr_id[j])


@pytest.mark.parametrize("name", ["sphere", "box", "perturbed"])
def test_series_and_per_node_forms_agree(bem, torch, oracle_lib, name):
    """The default series form (each pair's correction as a power series in kappa folded with
    the weights' moments) and the per-node form evaluate the same angular points: both match
    the oracle, and each other to rounding, for moments (two weight sets, complex nodes) and
    for the dense node combination."""
    xyz, tri = _mesh(name)
    n = len(tri)
    z, w, W = bem.contour_nodes(4.0, 1.5, 16, P=2)
    V = synth.probe_block(n, 16, seed=1)
    corr = _correction_ref(xyz, tri, 2.0, z, W, V)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Vd = _dev(torch, V)
        Cs = mesh.nearfield_moments(z, W, Vd).cpu().numpy()
        terms = mesh.nearfield_last_terms()
        Ss = mesh.assemble_sum(z, W[:, 0])
        mesh.nearfield_sum(z, W[:, 0], Ss)
        mesh.set_nearfield_mode(bem.NF_NODES)
        Cn = mesh.nearfield_moments(z, W, Vd).cpu().numpy()
        assert mesh.nearfield_last_terms() == 0
        Sn = mesh.assemble_sum(z, W[:, 0])
        mesh.nearfield_sum(z, W[:, 0], Sn)
        mesh.set_nearfield_mode(bem.NF_AUTO)
        Ss, Sn = Ss.cpu().numpy(), Sn.cpu().numpy()
        with pytest.raises(bem.BemError):
            mesh.set_nearfield_mode(2)
    assert terms in (12, 16, 24, 32), terms
    # error scale of either evaluation: sum_j |W[j, p]| |dT(z_j)| V, i.e. the p = 0 correction
    # (no cancellation among its nodes) times the ratio of the weight sums; set p = 1 cancels
    # to about 1e-5 of it, so its own norm is not the scale
    for p in range(2):
        ws = np.abs(W[:, p]).sum() / np.abs(W[:, 0]).sum()
        scale = ws * np.linalg.norm(Cn[0])
        e_sn = np.linalg.norm(Cs[p] - Cn[p]) / scale
        e_so = np.linalg.norm(Cs[p] - corr[p]) / scale
        print(f"{name} p={p}: {terms} terms; series vs per node {e_sn:.2e}, series vs oracle {e_so:.2e} "
              f"(|corr_p| / scale {np.linalg.norm(Cn[p]) / scale:.1e})")
        assert e_sn <= 1e-12 and e_so <= 1e-12
        # row by row, on the same scale per row
        rn = ws * np.linalg.norm(Cn[0], axis=1)
        assert np.all(np.linalg.norm(Cs[p] - Cn[p], axis=1) <= 1e-11 * rn + 1e-300)
    dS = Sn - Ss
    print(f"{name}: dense node combination, series vs per node {np.abs(dS).max() / np.abs(Sn).max():.2e}")
    assert np.abs(dS).max() <= 1e-13 * np.abs(Sn).max()


def test_series_form_falls_back_to_per_node_when_the_series_is_long(bem, torch, oracle_lib):
    """eta = 16 on the 80-triangle sphere: pairs span the whole surface, max |z| R_max is far
    beyond what 32 terms resolve, so the per-node form runs (and matches the oracle)."""
    xyz, tri = synth.perturbed_icosphere(1, 0.05, 9)
    n = len(tri)
    z = np.array([3.0 + 0.4j, 5.0 - 0.3j, 6.1 + 0.8j])
    W = np.array([[1.0], [0.5 - 0.2j], [0.3j]])
    V = synth.probe_block(n, 5, seed=3)
    corr = _correction_ref(xyz, tri, 16.0, z, W, V)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(16.0)
        Cg = mesh.nearfield_moments(z, W, _dev(torch, V)).cpu().numpy()
        assert mesh.nearfield_last_terms() == 0
    assert np.linalg.norm(Cg[0] - corr[0]) <= 1e-11 * np.linalg.norm(corr[0])


def test_no_list_leaves_moments_unchanged_and_errors(bem, torch):
    xyz, tri = synth.icosphere(2)
    n = len(tri)
    z, w, W = bem.contour_nodes(4.0, 1.5, 8, P=1)
    with bem.Mesh(xyz, tri) as mesh:
        Vd = _dev(torch, synth.probe_block(n, 4, seed=1))
        M0 = torch.ones((1, n, 4), dtype=torch.complex128, device="cuda")
        mesh.nearfield_moments(z, W, Vd, out=M0)
        assert bool((M0 == 1).all())
        mesh.set_nearfield(2.0)
        mesh.set_nearfield(0.0)  # removes the list again
        mesh.nearfield_moments(z, W, Vd, out=M0)
        assert bool((M0 == 1).all())
        for bad in (-1.0, 17.0, float("nan")):
            with pytest.raises(bem.BemError, match="EINVAL"):
                mesh.set_nearfield(bad)
        mesh.set_nearfield(2.0)
        with pytest.raises(bem.BemError, match="EINVAL"):
            mesh.nearfield_moments(z, np.full_like(W, np.nan), Vd, out=M0)
        torch.cuda.synchronize()


def test_deterministic(bem, torch):
    xyz, tri = synth.icosphere(3)
    z, w, W = bem.contour_nodes(5.0, 2.0, 24, P=2)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Vd = _dev(torch, synth.probe_block(len(tri), 8, seed=4))
        a = mesh.nearfield_moments(z, W, Vd)
        b = mesh.nearfield_moments(z, W, Vd)
        assert bool((a == b).all())


@pytest.mark.parametrize("eta,level", [(4.0, 2), (16.0, 1)])
def test_rows_longer_than_one_chunk(bem, torch, oracle_lib, eta, level):
    """Rows with more than 64 near pairs are taken in several chunks of different lengths
    (eta = 4: about 130 pairs per row, chunks of 64, 64 and the rest; eta = 16 on 80
    triangles: every other triangle is near, chunks of 64 and 15)."""
    xyz, tri = synth.perturbed_icosphere(level, 0.05, 9)
    n = len(tri)
    z = np.array([3.0 + 0.4j, 5.0 - 0.3j, 4.2, 6.1 + 0.8j, 2.5 + 0.1j, 3.3 - 0.9j])
    rng = np.random.default_rng(8)
    W = rng.normal(size=(6, 3)) + 1j * rng.normal(size=(6, 3))
    V = synth.probe_block(n, 7, seed=3)
    corr = _correction_ref(xyz, tri, eta, z, W, V)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(eta)
        rp, _ = mesh.nearfield_list()
        assert np.diff(rp).max() > 64
        Cg = mesh.nearfield_moments(z, W, _dev(torch, V)).cpu().numpy()
    for p in range(3):
        assert np.linalg.norm(Cg[p] - corr[p]) <= 1e-11 * np.linalg.norm(corr[p])


def test_single_node_weight_and_column(bem, torch, oracle_lib):
    xyz, tri = synth.icosphere(2)
    n = len(tri)
    z = np.array([4.5 + 0.2j])
    W = np.array([[0.7 - 0.3j]])
    V = synth.probe_block(n, 1, seed=6)
    corr = _correction_ref(xyz, tri, 2.0, z, W, V)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Cg = mesh.nearfield_moments(z, W, _dev(torch, V)).cpu().numpy()
    assert np.linalg.norm(Cg[0] - corr[0]) <= 1e-11 * np.linalg.norm(corr[0])


def test_nearfield_sum_matches_oracle(bem, torch, oracle_lib):
    """bem_assemble_sum + bem_nearfield_sum = sum_j c_j T_nf(z_j), the dense matrix of the
    corrected operator, against the oracle's dense corrected operators."""
    from oracle import method as M

    xyz, tri = synth.perturbed_icosphere(2, 0.05, 5)
    z, w, W = bem.contour_nodes(4.0, 1.5, 12, P=1)
    c = W[:, 0]
    op = M.Operator(xyz, tri, nearfield_eta=2.0)
    So = sum(c[j] * op.dense(z[j]) for j in range(len(z)))
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        S = mesh.assemble_sum(z, c)
        mesh.nearfield_sum(z, c, S)
        S = S.cpu().numpy()
    assert np.linalg.norm(S - So) <= TOL * np.linalg.norm(So)


def test_eigs_of_corrected_operator_match_golden(bem, torch, oracle_lib):
    """The Cauchy route on the corrected operator (every sweep, S, the projections and the
    residuals corrected) against the oracle's Algorithm 3 on the dense corrected operator:
    sphere-1280, |z - 4| < 1.5, N = 32, 16 probes (seed 1), eigenvalues to 1e-10."""
    import os

    from paper_1906_03938_amd.eig import eigs_in_contour

    gold = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "sphere1280_nearfield_eigs.txt"))
    lam_o = gold[:, 0] + 1j * gold[:, 1]
    xyz, tri = synth.icosphere(3)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        lam, X, res, outer = eigs_in_contour(mesh, 4.0, 1.5, 32, synth.probe_block(len(tri), 16, seed=1),
                                             nearfield=True)
    assert lam.size == lam_o.size and res.max() <= 1e-12
    for lo in lam_o:
        assert np.min(np.abs(lam - lo)) <= 1e-10 * abs(lo)


def test_interval_eigs_of_corrected_operator_match_golden(bem, torch, oracle_lib):
    """The Chebyshev route on the corrected operator (sweeps, G, restart blocks, projections
    and residuals corrected) against the oracle's Chebyshev route on the dense corrected
    operator: sphere-1280, kappa in [2.5, 5], N = 32, 16 probes (seed 1), eigenvalues to
    1e-10; the two golden files (Cauchy and Chebyshev routes) also agree with each other."""
    import os

    from paper_1906_03938_amd.eig import eigs_in_interval

    here = os.path.join(os.path.dirname(__file__), "golden")
    gold = np.loadtxt(os.path.join(here, "sphere1280_nearfield_interval_eigs.txt"))
    lam_o = gold[:, 0] + 1j * gold[:, 1]
    gold_c = np.loadtxt(os.path.join(here, "sphere1280_nearfield_eigs.txt"))
    for lo in gold_c[:, 0] + 1j * gold_c[:, 1]:
        assert np.min(np.abs(lam_o - lo)) <= 1e-10 * abs(lo)
    xyz, tri = synth.icosphere(3)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        lam, X, res, outer = eigs_in_interval(mesh, 2.5, 5.0, 32, synth.probe_block(len(tri), 16, seed=1),
                                              nearfield=True)
    assert lam.size == lam_o.size and res.max() <= 1e-12
    for lo in lam_o:
        assert np.min(np.abs(lam - lo)) <= 1e-10 * abs(lo)


def test_nearfield_project_matches_oracle(bem, torch, oracle_lib):
    """rr_project followed by bem_nearfield_project gives the projections U^H T_nf(z_j) U of
    the corrected operator: against the oracle's dense corrected operator (1e-12 per node, per
    row); rows of the per-node corrections are integrated only for the nodes of each chunk."""
    from oracle import method as M

    xyz, tri = synth.icosphere(3)
    op = M.Operator(xyz, tri, nearfield_eta=2.0)
    U, _ = np.linalg.qr(synth.probe_block(op.n, 8, seed=4))
    U = np.ascontiguousarray(U)
    s, w = M.circle_nodes(4.0, 1.5, 20)
    with bem.Mesh(xyz, tri) as mesh:
        mesh.set_nearfield(2.0)
        Ud = _dev(torch, U)
        P = mesh.rr_project(s, Ud)
        mesh.nearfield_project(s, Ud, P)
        P = P.cpu().numpy()
    Po = M.rr_project(op, s, U)
    for j in range(len(s)):
        e = np.linalg.norm(P[j] - Po[j]) / np.linalg.norm(Po[j])
        er = np.max(np.linalg.norm(P[j] - Po[j], axis=1) / np.linalg.norm(Po[j], axis=1))
        assert e <= TOL and er <= TOL, (j, e, er)

