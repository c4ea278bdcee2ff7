"""GPU parity of the reduced-precision forms (FP64 generation, FP32 / BF16 / FP16 matrix-core
contraction with FP32 accumulation, FP64 self terms) against the FP64 oracle on the
sphere-1280 workload.

Tolerances, normwise relative per node or weight set, from the arithmetic: every entry and
every probe value is rounded once to the contraction type (relative error <= u), the
products' errors have independent signs, so a sum of n products carries a relative error
of about u (observed 0.5-0.7 u for BF16 and FP16); FP32 sums additionally accumulate in
FP32, about sqrt(n) u more (observed ~12 u at n = 1280).  The tests allow 2 u for BF16 /
FP16 and 40 u for FP32, with u = 2^-8 (BF16), 2^-11 (FP16), 2^-24 (FP32)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

U_ROUND = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
FACTOR = {"f32": 40.0, "bf16": 2.0, "f16": 2.0}


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1906_03938_amd as bem
    from oracle import method as M

    assert torch.cuda.is_available()
    xyz, tri = synth.icosphere(3)
    op = M.Operator(xyz, tri)
    mesh = bem.Mesh(xyz, tri)
    V = synth.probe_block(op.n, 16, seed=1)
    yield bem, M, torch, mesh, op, V, torch.from_numpy(V).to("cuda")
    mesh.close()


def _prec(bem, name):
    return {"f32": bem.PREC_F32, "bf16": bem.PREC_BF16, "f16": bem.PREC_F16}[name]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["f32", "bf16", "f16"])
def test_contour_moments_and_projections(ctx, prec):
    """Complex nodes: AUTO takes the direct form at reduced precision."""
    bem, M, torch, mesh, op, V, Vd = ctx
    tol = FACTOR[prec] * U_ROUND[prec]
    s, w = M.circle_nodes(4.0, 1.5, 32)
    W = M.moment_weights(s, w, 4.0, 2)
    Mg = mesh.contour_moments(s, W, Vd, form=bem.FORM_AUTO | _prec(bem, prec)).cpu().numpy()
    assert mesh.last_form()[0] == bem.FORM_DIRECT
    Mo = M.contour_moments(op, s, W, V)
    errs = [_rel(Mg[p], Mo[p]) for p in range(2)]
    U, _ = np.linalg.qr(V)
    U = np.ascontiguousarray(U)
    P = mesh.rr_project(s[:6], torch.from_numpy(U).to("cuda"), form=bem.FORM_AUTO | _prec(bem, prec)).cpu().numpy()
    Po = M.rr_project(op, s[:6], U)
    errs += [_rel(P[j], Po[j]) for j in range(6)]
    print(prec, "moments/projections max rel err", max(errs), "tol", tol, flush=True)
    assert max(errs) <= tol


@pytest.mark.parametrize("prec", ["f32", "bf16", "f16"])
def test_cheb_moments(ctx, prec):
    """Real nodes: AUTO takes the Chebyshev (Jacobi-Anger) form at reduced precision."""
    bem, M, torch, mesh, op, V, Vd = ctx
    tol = FACTOR[prec] * U_ROUND[prec]
    a, b, N, L = 2.5, 5.5, 24, 20
    C = mesh.cheb_moments(a, b, N, L, Vd, form=bem.FORM_AUTO | _prec(bem, prec)).cpu().numpy()
    assert mesh.last_form()[0] == bem.FORM_CHEB
    Co = M.cheb_moments(op, a, b, N, L, V)
    err = max(np.linalg.norm(C[l] - Co[l]) for l in range(L)) / np.linalg.norm(Co[0])
    print(prec, "chebyshev blocks max err / |C_0|", err, "tol", tol, flush=True)
    assert err <= tol


@pytest.mark.parametrize("prec", ["f32", "bf16", "f16"])
def test_assemble_apply_and_ragged(ctx, prec):
    """Direct products, and a ragged open subset (n = 777, m = 33) that leaves partial row,
    column and operator blocks."""
    bem, M, torch, mesh, op, V, Vd = ctx
    tol = FACTOR[prec] * U_ROUND[prec]
    ks = np.array([4.0, 5.5 - 1.5j, 2.5 + 1.0j])
    Y = mesh.assemble_apply(ks, Vd, form=bem.FORM_DIRECT | _prec(bem, prec)).cpu().numpy()
    errs = [_rel(Y[j], op.apply(ks[j], V)) for j in range(3)]
    xyz, tri = synth.icosphere(3)
    keep = tri[:777]
    used = np.unique(keep)
    remap = -np.ones(xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    xyz2, tri2 = xyz[used], remap[keep].astype(np.int32)
    op2 = M.Operator(xyz2, tri2)
    V2 = synth.probe_block(777, 33, seed=4)
    with bem.Mesh(xyz2, tri2) as m2:
        Y2 = m2.assemble_apply([4.5 + 0.2j], torch.from_numpy(V2).to("cuda"),
                               form=bem.FORM_DIRECT | _prec(bem, prec)).cpu().numpy()
    errs.append(_rel(Y2[0], op2.apply(4.5 + 0.2j, V2)))
    print(prec, "apply max rel err", max(errs), "tol", tol, flush=True)
    assert max(errs) <= tol


def test_unknown_precision_is_rejected(ctx):
    bem, M, torch, mesh, op, V, Vd = ctx
    from paper_1906_03938_amd import _lib

    with pytest.raises(bem.BemError) as e:
        mesh.assemble_apply([4.0], Vd, form=0x40)
    assert e.value.status == _lib.BEM_EUNSUPPORTED
