"""contour_moments_noalloc, the allocation-free entry point (workspace in the library's static
scratch array), against contour_moments on the same inputs: calls in a row on one device, each
smaller than the first, in the unfolded FP64 route (generated products in the scratch), the
folded route (fold widths 2 and 4) and a reduced-precision sweep; the results are bitwise equal (same kernels, same order).
Device free memory is unchanged across a call on a fresh handle, and a call whose workspace
exceeds the array is rejected before anything is launched, leaving its output untouched."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _case(bem, torch, level, N, P, m, seed, flags):
    xyz, tri = synth.icosphere(level)
    n = tri.shape[0]
    z, _, W = bem.contour_nodes(4.0, 1.5, N, P=P)
    V = torch.from_numpy(synth.probe_block(n, m, seed=seed)).to("cuda")
    return xyz, tri, z, W, V


@pytest.mark.parametrize("flags_name", ["f64", "f32"])
def test_noalloc_equals_contour_moments(flags_name):
    import torch

    import paper_1906_03938_amd as bem

    prec = bem.PREC_F64 if flags_name == "f64" else bem.PREC_F32
    # (level, N, P, m): an unfolded call (P = 9 > 4 weight sets, Z in the scratch), then
    # smaller folded ones (fold widths 2 and 4, the second padded for P = 3)
    for level, N, P, m, seed in ((4, 32, 9, 16, 1), (3, 16, 2, 8, 2), (3, 16, 3, 5, 5)):
        xyz, tri, z, W, V = _case(bem, torch, level, N, P, m, seed, prec)
        print(f"case n={tri.shape[0]} N={N} P={P} m={m} {flags_name}", flush=True)
        with bem.Mesh(xyz, tri) as mesh:
            ref = mesh.contour_moments(z, W, V, form=bem.FORM_AUTO | prec)
            out = torch.full((P, tri.shape[0], m), float("nan"), dtype=torch.complex128, device="cuda")
            mesh.contour_moments_noalloc(z, W, V, out=out, form=bem.FORM_AUTO | prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)


def test_noalloc_allocates_nothing_and_rejects_oversize():
    import torch

    import paper_1906_03938_amd as bem

    xyz, tri, z, W, V = _case(bem, torch, 4, 32, 9, 16, 3, 0)
    out = torch.zeros((9, tri.shape[0], 16), dtype=torch.complex128, device="cuda")
    with bem.Mesh(xyz, tri) as warm:  # loads the code object, warms the runtime
        warm.contour_moments_noalloc(z, W, V, out=out)
    torch.cuda.synchronize()
    with bem.Mesh(xyz, tri) as mesh:
        torch.cuda.synchronize()
        before = _free_bytes()
        mesh.contour_moments_noalloc(z, W, V, out=out)
        torch.cuda.synchronize()
        after = _free_bytes()
        print(f"free bytes before {before}, after {after}", flush=True)
        assert after == before
        ref = mesh.contour_moments(z, W, V)  # the handle's workspace is allocated on this call
        assert torch.equal(out, ref)
    # a call that needs more than the scratch array: rejected, output untouched
    xyz, tri, z, W, V = _case(bem, torch, 5, 32, 9, 64, 4, 0)
    with bem.Mesh(xyz, tri) as mesh:
        big = torch.full((9, tri.shape[0], 64), 7.0, dtype=torch.complex128, device="cuda")
        with pytest.raises(bem.BemError, match="EINVAL"):
            mesh.contour_moments_noalloc(z, W, V, out=big)
        torch.cuda.synchronize()
        assert bool((big == 7.0).all())
