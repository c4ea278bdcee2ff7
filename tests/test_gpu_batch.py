"""GPU tests of the batched persistent form (several meshes, each with its own contour, in
one generate-and-contract launch): parity with the oracle's per-mesh contour moments
(1e-12 normwise per mesh and weight set), bitwise equality with the per-mesh entry point
in the same form (the tiles run the same arithmetic in the same order, whatever the column
tile the autotuner picks; up to four weight sets folded into the sweep as contour_moments
does, more contracted per operator and recombined as rr_project's fused moments are), graph
capture and replay, error paths, and sampled-row parity
on the full 64-ellipsoid workload (geodesic frequencies 10..44, 2,000-38,720 triangles
per mesh, circles |z - c_i| = 1 with c_i in [3, 7], N = 32, m = 32, seed 4)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small():
    """Five ellipsoids of 180-980 triangles (frequencies 3..7), N = 16, P = 2, m = 20."""
    import torch

    import paper_1906_03938_amd as bem

    assert torch.cuda.is_available()
    spec = synth.ellipsoid_batch(count=5, seed=5, freq=(3, 7))
    meshes = [bem.Mesh(x, t) for x, t, _, _ in spec]
    N, P, m = 16, 2, 20
    z, W = [], []
    for _, _, _, c in spec:
        zi, _, Wi = bem.contour_nodes(c, 1.0, N, P=P)
        z.append(zi)
        W.append(Wi)
    V = [synth.probe_block(t.shape[0], m, seed=10 + i) for i, (_, t, _, _) in enumerate(spec)]
    yield bem, torch, spec, meshes, np.array(z), np.array(W), V, N, P, m
    for mm in meshes:
        mm.close()


def _packed(torch, V):
    return torch.from_numpy(np.ascontiguousarray(np.concatenate(V, axis=0))).to("cuda")


@pytest.mark.parametrize("form", ["auto", "direct", "expand"])
def test_batch_matches_oracle(small, form):
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    from oracle import method as M

    f = {"auto": bem.FORM_AUTO, "direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND}[form]
    with bem.Batch(meshes, z, W, m, form=f) as b:
        assert list(np.diff(b.rows)) == [t.shape[0] for _, t, _, _ in spec]
        if form != "auto":
            assert b.form == f
        Mg = [x.cpu().numpy() for x in b.split(b.moments(_packed(torch, V)))]
        print(form, "form used", b.form, "operators", b.operators, "col tile", b.col_tile, flush=True)
    errs = []
    for i, (x, t, _, c) in enumerate(spec):
        op = M.Operator(x, t)
        zo, wo = M.circle_nodes(c, 1.0, N)
        Mo = M.contour_moments(op, zo, M.moment_weights(zo, wo, c, P), V[i])
        errs += [_rel(Mg[i][p], Mo[p]) for p in range(P)]
    print(form, "max rel err", max(errs), flush=True)
    assert max(errs) <= TOL


@pytest.mark.parametrize("form", ["direct", "expand"])
@pytest.mark.parametrize("tune", [False, True])
def test_batch_bitwise_equals_per_mesh(small, form, tune):
    """Two weight sets: the batch folds them into the sweep, as contour_moments does per mesh
    (the same folded tiles, whatever column tile the autotuner picks)."""
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND}[form]
    with bem.Batch(meshes, z, W, m, form=f, tune=tune) as b:
        Mb = b.split(b.moments(_packed(torch, V)))
        print(form, "tune", tune, "col tile", b.col_tile, flush=True)
        for i, mesh in enumerate(meshes):
            Mi = mesh.contour_moments(z[i], W[i], torch.from_numpy(V[i]).to("cuda"), form=f)
            assert mesh.last_form()[0] == b.form and mesh.last_form()[1] == b.operators[i]
            assert torch.equal(Mi, Mb[i]), i


def _weights(bem, spec, N, P):
    z, W = [], []
    for _, _, _, c in spec:
        zi, _, Wi = bem.contour_nodes(c, 1.0, N, P=P)
        z.append(zi)
        W.append(Wi)
    return np.array(z), np.array(W)


@pytest.mark.parametrize("form", ["direct", "expand"])
@pytest.mark.parametrize("P", [3, 4])
def test_batch_folds_four_weight_sets_bitwise(small, form, P):
    """Three or four weight sets: the batch folds them at width 4 (the P = 3 coefficient rows
    padded with a zero column), as contour_moments does per mesh, bitwise equal to it and
    within the oracle's tolerance."""
    bem, torch, spec, meshes, z, W, V, N, _, m = small
    from oracle import method as M

    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND}[form]
    zP, WP = _weights(bem, spec, N, P)
    with bem.Batch(meshes, zP, WP, m, form=f) as b:
        Mb = b.split(b.moments(_packed(torch, V)))
        for i, mesh in enumerate(meshes):
            Mi = mesh.contour_moments(zP[i], WP[i], torch.from_numpy(V[i]).to("cuda"), form=f)
            assert mesh.last_form()[0] == b.form and mesh.last_form()[1] == b.operators[i]
            assert torch.equal(Mi, Mb[i]), i
            x, t, _, c = spec[i]
            zo, wo = M.circle_nodes(c, 1.0, N)
            Mo = M.contour_moments(M.Operator(x, t), zo, M.moment_weights(zo, wo, c, P), V[i])
            for q in range(P):
                assert _rel(Mb[i][q].cpu().numpy(), Mo[q]) <= TOL, (i, q)


@pytest.mark.parametrize("form", ["direct", "expand"])
def test_batch_unfolded_bitwise_equals_per_mesh(small, form):
    """Five weight sets: the batch contracts every operator and recombines, as rr_project's
    fused moments do per mesh (the same sweep tiles and recombination), and matches the
    oracle."""
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    from oracle import method as M

    f = {"direct": bem.FORM_DIRECT, "expand": bem.FORM_EXPAND}[form]
    z5, W5 = _weights(bem, spec, N, 5)
    with bem.Batch(meshes, z5, W5, m, form=f) as b:
        Mb = b.split(b.moments(_packed(torch, V)))
        for i, mesh in enumerate(meshes):
            _, Mi = mesh.rr_project(z5[i], torch.from_numpy(V[i]).to("cuda"), W=W5[i], form=f)
            assert torch.equal(Mi, Mb[i]), i
            x, t, _, c = spec[i]
            zo, wo = M.circle_nodes(c, 1.0, N)
            Mo = M.contour_moments(M.Operator(x, t), zo, M.moment_weights(zo, wo, c, 5), V[i])
            for q in range(5):
                assert _rel(Mb[i][q].cpu().numpy(), Mo[q]) <= TOL, (i, q)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_graph_capture_replays(small, prec):
    """The moments call only launches kernels (at reduced precision also the per-mesh probe
    scale reductions, cleared by a kernel): captured once, every replay (with other work and
    synchronisations in between) reproduces the eager result bitwise."""
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    flags = bem.FORM_AUTO | (bem.PREC_F32 if prec == "f32" else bem.PREC_F64)
    with bem.Batch(meshes, z, W, m, form=flags) as b:
        Vd = _packed(torch, V)
        ref = b.moments(Vd).clone()
        out = torch.empty_like(ref)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            b.moments(Vd, out=out)  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            b.moments(Vd, out=out)
        for rep in range(3):
            out.zero_()
            meshes[0].contour_moments(z[0], W[0], torch.from_numpy(V[0]).to("cuda"))  # unrelated eager work
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), rep


U_ROUND = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
U_FACTOR = {"f32": 40.0, "bf16": 2.0, "f16": 2.0}  # as for the per-mesh reduced-precision calls


@pytest.mark.parametrize("prec", ["f32", "bf16", "f16"])
def test_batch_reduced_precision(small, prec):
    """Reduced-precision batch (AUTO = direct form): bitwise equal to the per-mesh calls at the
    same arithmetic (same tiles, same per-mesh probe scale), and within the arithmetic's
    tolerance of the oracle."""
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    from oracle import method as M

    p = {"f32": bem.PREC_F32, "bf16": bem.PREC_BF16, "f16": bem.PREC_F16}[prec]
    with bem.Batch(meshes, z, W, m, form=bem.FORM_AUTO | p) as b:
        assert b.form == bem.FORM_DIRECT
        Mb = b.split(b.moments(_packed(torch, V)))
        print(prec, "col tile", b.col_tile, "operators", b.operators, flush=True)
        errs = []
        for i, (x, t, _, c) in enumerate(spec):
            Mi = meshes[i].contour_moments(z[i], W[i], torch.from_numpy(V[i]).to("cuda"), form=bem.FORM_AUTO | p)
            assert torch.equal(Mi, Mb[i]), i
            op = M.Operator(x, t)
            zo, wo = M.circle_nodes(c, 1.0, N)
            Mo = M.contour_moments(op, zo, M.moment_weights(zo, wo, c, P), V[i])
            errs += [_rel(Mb[i][q].cpu().numpy(), Mo[q]) for q in range(P)]
    print(prec, "max rel err vs oracle", max(errs), flush=True)
    assert max(errs) <= U_FACTOR[prec] * U_ROUND[prec]


def test_batch_reduced_precision_tuned_expand(small):
    """FP32 with the expansion form on request and the autotuned column tile: still bitwise
    equal to the per-mesh calls in that form."""
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    f = bem.FORM_EXPAND | bem.PREC_F32
    with bem.Batch(meshes, z, W, m, form=f, tune=True) as b:
        assert b.form == bem.FORM_EXPAND
        Mb = b.split(b.moments(_packed(torch, V)))
        print("f32 expand col tile", b.col_tile, flush=True)
        for i in range(len(meshes)):
            _, Mi = meshes[i].rr_project(z[i], torch.from_numpy(V[i]).to("cuda"), W=W[i], form=f)
            assert torch.equal(Mi, Mb[i]), i


def test_batch_error_paths(small):
    bem, torch, spec, meshes, z, W, V, N, P, m = small
    from paper_1906_03938_amd import _lib

    for flags in (bem.FORM_CHEB, bem.FORM_CHEB | bem.PREC_F32, bem.FORM_AUTO | 0x40):
        with pytest.raises(bem.BemError) as e:
            bem.Batch(meshes, z, W, m, form=flags)
        assert e.value.status == _lib.BEM_EUNSUPPORTED
    bad = z.copy()
    bad[1, 3] = np.nan
    with pytest.raises(bem.BemError) as e:
        bem.Batch(meshes, bad, W, m)
    assert e.value.status == _lib.BEM_EINVAL
    with bem.Batch(meshes, z, W, m) as b:
        with pytest.raises(ValueError):
            b.moments(torch.zeros((int(b.rows[-1]) + 1, m), dtype=torch.complex128, device="cuda"))


def test_batch_ellipsoids64_sampled_rows():
    """The full 64-ellipsoid workload: sampled target rows of the smallest and the largest
    mesh (and one in between) against the oracle, row by row."""
    import torch

    import paper_1906_03938_amd as bem
    from oracle import method as M

    assert torch.cuda.is_available()
    spec = synth.ellipsoid_batch()
    sizes = np.array([t.shape[0] for _, t, _, _ in spec])
    assert sizes.min() >= 2000 and sizes.max() <= 38720 and len(spec) == 64
    N, P, m = 32, 2, 32
    meshes = [bem.Mesh(x, t) for x, t, _, _ in spec]
    z, W = [], []
    for _, _, _, c in spec:
        zi, _, Wi = bem.contour_nodes(c, 1.0, N, P=P)
        z.append(zi)
        W.append(Wi)
    V = [synth.probe_block(int(n), m, seed=4000 + i) for i, n in enumerate(sizes)]
    with bem.Batch(meshes, np.array(z), np.array(W), m) as b:
        b.set_timing(True)
        Mb = b.moments(torch.from_numpy(np.concatenate(V, axis=0)).to("cuda"))
        ms = b.last_kernel_ms()
        parts = b.split(Mb)
        print(f"form {b.form}, col tile {b.col_tile}, persistent kernel {ms:.1f} ms", flush=True)
        for i in (int(sizes.argmin()), int(sizes.argmax()), 7):
            x, t, _, c = spec[i]
            n = t.shape[0]
            rows = np.unique(np.array([0, 1, n // 3, n // 2 + 5, n - 2, n - 1]))
            op = M.Operator(x, t)
            zo, wo = M.circle_nodes(c, 1.0, N)
            Mo = M.contour_moments(op, zo, M.moment_weights(zo, wo, c, P), V[i], rows=rows)
            Mg = parts[i].cpu().numpy()[:, rows]
            for p in range(P):
                e = _rel(Mg[p], Mo[p])
                print(f"mesh {i} (n = {n}) moment {p + 1}: rel err {e:.2e}", flush=True)
                assert e <= TOL
    for mm in meshes:
        mm.close()


@pytest.mark.parametrize("m", [1, 33])
def test_batch_edge_shapes(m):
    """A batch mixing the 20-triangle icosahedron (one row block, mostly padding), a ragged
    open subset (n = 777) and one of the small ellipsoids, with a single probe column and
    with a ragged column count: bitwise equal to the per-mesh calls and to the oracle."""
    import torch

    import paper_1906_03938_amd as bem
    from oracle import method as M

    x0, t0 = synth.icosahedron()
    xs, ts = synth.icosphere(3)
    keep = ts[:777]
    used = np.unique(keep)
    remap = -np.ones(xs.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    x1, t1 = xs[used], remap[keep].astype(np.int32)
    x2, t2, _, _ = synth.ellipsoid_batch(count=1, seed=9, freq=(4, 4))[0]
    geo = [(x0, t0, 4.0), (x1, t1, 4.5), (x2, t2, 3.5)]
    meshes = [bem.Mesh(x, t) for x, t, _ in geo]
    N, P = 12, 2
    z, W = [], []
    for _, _, c in geo:
        zi, _, Wi = bem.contour_nodes(c, 1.0, N, P=P)
        z.append(zi)
        W.append(Wi)
    V = [synth.probe_block(t.shape[0], m, seed=50 + i) for i, (_, t, _) in enumerate(geo)]
    try:
        with bem.Batch(meshes, np.array(z), np.array(W), m) as b:
            Mb = b.split(b.moments(torch.from_numpy(np.concatenate(V)).to("cuda")))
            for i, (x, t, c) in enumerate(geo):
                Mi = meshes[i].contour_moments(z[i], W[i], torch.from_numpy(V[i]).to("cuda"), form=b.form)
                assert torch.equal(Mi, Mb[i]), i
                op = M.Operator(x, t)
                zo, wo = M.circle_nodes(c, 1.0, N)
                Mo = M.contour_moments(op, zo, M.moment_weights(zo, wo, c, P), V[i])
                for q in range(P):
                    assert _rel(Mb[i][q].cpu().numpy(), Mo[q]) <= TOL, (i, q)
    finally:
        for mm in meshes:
            mm.close()
