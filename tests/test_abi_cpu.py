"""CPU checks of the C ABI: the library loads, exports every declared entry point, its
host-side node and weight generators match the oracle's, and host-side argument
validation rejects bad calls before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1906_03938_amd as bem
from paper_1906_03938_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bemrat.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"defined"})


def test_library_exports_every_declared_symbol():
    L = bem.lib()
    names = _declared()
    assert set(_lib.EXPORTS) == set(names), names
    for name in names:
        assert hasattr(L, name), name


def test_contour_nodes_match_oracle(oracle_lib):
    from oracle import method as M

    for c, R, N, P in ((4.0, 1.5, 32, 3), (5.0 + 0.5j, 2.0, 64, 5), (-1j, 0.3, 7, 1)):
        z, w, W = bem.contour_nodes(c, R, N, P=P)
        zo, wo = M.circle_nodes(c, R, N)
        Wo = M.moment_weights(zo, wo, c, P)
        assert np.abs(z - zo).max() <= 4e-16 * (abs(c) + R)
        assert np.abs(w - wo).max() <= 4e-16 * R
        assert np.abs(W - Wo).max() <= 1e-14 * np.abs(Wo).max()


def test_cheb_nodes_match_oracle(oracle_lib):
    from oracle import method as M

    for a, b, N in ((2.0, 8.0, 48), (3.0, 8.0, 25), (-1.0, 1.0, 1)):
        k, coef = bem.cheb_nodes(a, b, N)
        ko, co = M.cheb_nodes(a, b, N)
        assert np.abs(k - ko).max() <= 4e-16 * max(abs(a), abs(b))
        assert np.abs(coef - co).max() <= 1e-15


def test_host_argument_errors():
    with pytest.raises(bem.BemError) as e:
        bem.contour_nodes(4.0, -1.0, 8)
    assert e.value.status == _lib.BEM_EINVAL
    with pytest.raises(bem.BemError):
        bem.contour_nodes(4.0, 1.0, 0)
    with pytest.raises(bem.BemError):
        bem.cheb_nodes(3.0, 2.0, 8)
    with pytest.raises(bem.BemError):
        bem.cheb_nodes(float("nan"), 2.0, 8)
    L = bem.lib()
    # null handles are rejected before any device call
    assert L.bem_mesh_size(None) == -1
    assert L.bem_last_form(None, None, None) == _lib.BEM_EINVAL
    assert L.bem_set_timing(None, 1) == _lib.BEM_EINVAL
    k = np.zeros(2)
    assert L.bem_assemble_apply(None, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1, None, 1, 1, None, 1, 0,
                                None) == _lib.BEM_EINVAL
    assert L.rr_project(None, None, 1, None, 1, 1, None, None, 0, None, 1, 0, None) == _lib.BEM_EINVAL
    out = ctypes.c_void_p(123)
    assert L.bem_mesh_create(None, 3, None, 1, None, ctypes.byref(out)) == _lib.BEM_EINVAL
    assert out.value is None
    assert b"NULL" in L.bem_last_error()


def test_mesh_validation_before_device():
    """Index errors and non-finite coordinates are found on the host."""
    L = bem.lib()
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float64)
    tri = np.array([[0, 1, 3]], dtype=np.int32)
    out = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    assert L.bem_mesh_create(xyz.ctypes.data_as(dp), 3, tri.ctypes.data_as(ip), 1, None,
                             ctypes.byref(out)) == _lib.BEM_EMESH
    xyz[1, 1] = np.inf
    tri[0, 2] = 2
    assert L.bem_mesh_create(xyz.ctypes.data_as(dp), 3, tri.ctypes.data_as(ip), 1, None,
                             ctypes.byref(out)) == _lib.BEM_EINVAL
