"""GPU parity at the full headline size, workload "sphere-81920": unit icosphere level 6
(n = 81920), circle |z - 5| = 2 with N = 64 nodes, m = 64 probes (seed 2) -- the call
bench.py times (rr_project with 2 fused moments, automatic form).  The oracle evaluates
sampled target rows one by one; quantities that need every row (the projections) are
checked through the identity P_j = U^H Y_j against per-node products Y_j that are
themselves checked on the sampled rows.  Also the Chebyshev blocks on [2, 8] with N = 48.
Tolerance: 1e-12 normwise per node / weight set over the sampled rows."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
ROWS = np.array([0, 1, 777, 20480, 40961, 65535, 81918, 81919], dtype=np.int64)


@pytest.fixture(scope="module")
def big():
    import torch

    import paper_1906_03938_amd as bem
    from oracle import method as M

    assert torch.cuda.is_available()
    xyz, tri = synth.icosphere(6)
    V = synth.probe_block(tri.shape[0], 64, seed=2)
    mesh = bem.Mesh(xyz, tri)
    yield bem, M, torch, mesh, M.Operator(xyz, tri), V, torch.from_numpy(V).to("cuda")
    mesh.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_rr_project_and_moments_at_scale(big):
    bem, M, torch, mesh, op, V, Vd = big
    z, w, W = bem.contour_nodes(5.0, 2.0, 64, P=2)
    P, Mg = mesh.rr_project(z, Vd, W=W)
    used, L = mesh.last_form()
    print(f"form {used} with {L} generated operators", flush=True)
    Mg = Mg.cpu().numpy()[:, ROWS]
    zo, wo = M.circle_nodes(5.0, 2.0, 64)
    Wo = M.moment_weights(zo, wo, 5.0, 2)
    Mo = M.contour_moments(op, zo, Wo, V, rows=ROWS)
    for p in range(2):
        e = _rel(Mg[p], Mo[p])
        print(f"moment {p + 1}: rel err {e:.2e}", flush=True)
        assert e <= TOL
    # per-node products (direct form) on sampled rows, and P_j = U^H Y_j
    sel = [0, 21, 47]
    Y = mesh.assemble_apply(z[sel], Vd)
    Yh = Y.cpu().numpy()[:, ROWS]
    for t, j in enumerate(sel):
        e = _rel(Yh[t], op.apply(zo[j], V, rows=ROWS))
        print(f"node {j}: rel err {e:.2e}", flush=True)
        assert e <= TOL
        Pj = (Vd.conj().T @ Y[t]).cpu().numpy()
        e = _rel(P[j].cpu().numpy(), Pj)
        print(f"projection {j}: rel err vs U^H Y {e:.2e}", flush=True)
        assert e <= TOL


def test_cheb_moments_at_scale(big):
    bem, M, torch, mesh, op, V, Vd = big
    a, b, N, L = 2.0, 8.0, 48, 48
    C = mesh.cheb_moments(a, b, N, L, Vd).cpu().numpy()[:, ROWS]
    Co = M.cheb_moments(op, a, b, N, L, V, rows=ROWS)
    scale = np.linalg.norm(Co[0])
    err = max(np.linalg.norm(C[l] - Co[l]) for l in range(L)) / scale
    print(f"chebyshev blocks: max error / |C_0| = {err:.2e}", flush=True)
    assert err <= TOL
