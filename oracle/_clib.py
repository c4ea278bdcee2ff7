"""ctypes loader and thin wrappers for the oracle's C core (bem_oracle.c).

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the benchmark's CPU
baseline leg.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def build(verbose: bool = False) -> str:
    """Compiles bem_oracle.c into liboracle.so (gcc, -O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_radon7.argtypes = [_dp, _dp]
        L.or_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
        L.or_geometry.argtypes = [_dp, _i64, _i32p, _i64, _dp, _dp, _dp, _dp]
        L.or_geometry.restype = ctypes.c_int
        L.or_self_term_tri.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
        L.or_self_terms.argtypes = [_dp, _i64, _i32p, _i64, _dp, _i64, ctypes.c_int, _dp]
        L.or_self_terms.restype = ctypes.c_int
        L.or_dense.argtypes = [_dp, _i64, _i32p, _i64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, _dp]
        L.or_dense.restype = ctypes.c_int
        L.or_apply_rows.argtypes = [_dp, _i64, _i32p, _i64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, _i64p, _i64, _dp, _i64, _i64, _dp]
        L.or_apply_rows.restype = ctypes.c_int
        L.or_num_threads.restype = ctypes.c_int
        L.or_tri_integral.argtypes = [_dp, _dp, _dp, _i64, ctypes.c_double, _dp]
        L.or_tri_integral.restype = ctypes.c_int
        L.or_near_pairs.argtypes = [_dp, _i64, _i32p, _i64, ctypes.c_double, _i64p, _i32p, _i64]
        L.or_near_pairs.restype = ctypes.c_int64
        L.or_nearfield_correction.argtypes = [_dp, _i64, _i32p, _i64, _i64p, _i32p, _dp, _i64,
                                              ctypes.c_double, _dp]
        L.or_nearfield_correction.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _check(rc: int):
    if rc != 0:
        raise ValueError({-1: "triangle index out of range", -2: "degenerate triangle",
                          -3: "allocation failure"}.get(rc, f"oracle error {rc}"))


def _mesh(xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return xyz, tri


def radon7():
    b = np.zeros((7, 3))
    w = np.zeros(7)
    lib().or_radon7(_d(b), _d(w))
    return b, w


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().or_gauss_legendre(n, _d(x), _d(w))
    return x, w


def geometry(xyz, tri):
    xyz, tri = _mesh(xyz, tri)
    n = tri.shape[0]
    area = np.zeros(n)
    cen = np.zeros((n, 3))
    qp = np.zeros((n, 7, 3))
    qw = np.zeros((n, 7))
    _check(lib().or_geometry(_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n,
                             _d(area), _d(cen), _d(qp), _d(qw)))
    return area, cen, qp, qw


def self_term_tri(P, kappa, deriv: int = 0) -> complex:
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    out = np.zeros(2)
    k = complex(kappa)
    lib().or_self_term_tri(_d(P), k.real, k.imag, int(deriv), _d(out))
    return complex(out[0], out[1])


def self_terms(xyz, tri, kappas, deriv: int = 0) -> np.ndarray:
    """nk x n complex: T_aa(kappa_j)."""
    xyz, tri = _mesh(xyz, tri)
    k = np.ascontiguousarray(np.atleast_1d(np.asarray(kappas, dtype=np.complex128)))
    n = tri.shape[0]
    out = np.zeros((k.size, n), dtype=np.complex128)
    _check(lib().or_self_terms(_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n,
                               k.view(np.float64).ctypes.data_as(_dp), k.size, int(deriv),
                               out.view(np.float64).ctypes.data_as(_dp)))
    return out


def dense(xyz, tri, kappa, deriv: int = 0) -> np.ndarray:
    """Dense T(kappa) (or its deriv-th derivative in kappa), n x n complex."""
    xyz, tri = _mesh(xyz, tri)
    n = tri.shape[0]
    T = np.zeros((n, n), dtype=np.complex128)
    k = complex(kappa)
    _check(lib().or_dense(_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n, k.real, k.imag,
                          int(deriv), T.view(np.float64).ctypes.data_as(_dp)))
    return T


def apply_rows(xyz, tri, kappa, V, rows=None, deriv: int = 0) -> np.ndarray:
    """Rows `rows` of T(kappa) @ V, matrix-free with compensated summation."""
    xyz, tri = _mesh(xyz, tri)
    n = tri.shape[0]
    V = np.ascontiguousarray(V, dtype=np.complex128)
    if V.ndim == 1:
        V = V[:, None]
    if V.shape[0] != n:
        raise ValueError("V must have n rows")
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = V.shape[1]
    Y = np.zeros((rows.size, m), dtype=np.complex128)
    k = complex(kappa)
    _check(lib().or_apply_rows(_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n, k.real,
                               k.imag, int(deriv), rows.ctypes.data_as(_i64p), rows.size,
                               V.view(np.float64).ctypes.data_as(_dp), m, m,
                               Y.view(np.float64).ctypes.data_as(_dp)))
    return Y


def num_threads() -> int:
    return int(lib().or_num_threads())


def tri_integral(x, P, kappas, rtol: float = 1e-15) -> np.ndarray:
    """Adaptive integral of exp(i k |x - y|)/(4 pi |x - y|) over triangle P (3 x 3), one
    value per wavenumber."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    k = np.ascontiguousarray(np.atleast_1d(np.asarray(kappas, dtype=np.complex128)))
    out = np.zeros(k.size, dtype=np.complex128)
    _check(lib().or_tri_integral(_d(x), _d(P), k.view(np.float64).ctypes.data_as(_dp), k.size,
                                 float(rtol), out.view(np.float64).ctypes.data_as(_dp)))
    return out


def near_pairs(xyz, tri, eta: float):
    """Near-pair list (rowptr[n + 1], col[nnz]) by brute force over all pairs."""
    xyz, tri = _mesh(xyz, tri)
    n = tri.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    args = (_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n, float(eta), rowptr.ctypes.data_as(_i64p))
    cnt = lib().or_near_pairs(*args, None, 0)
    _check(int(min(cnt, 0)))
    col = np.zeros(max(cnt, 1), dtype=np.int32)
    cnt2 = lib().or_near_pairs(*args, col.ctypes.data_as(_i32p), col.size)
    _check(int(min(cnt2, 0)))
    return rowptr, col[:cnt]


def nearfield_correction(xyz, tri, eta: float, kappas, rtol: float = 1e-15):
    """(rowptr, col, dT): the near-pair list and dT[j, i] = integral - 7-point value of pair
    i at wavenumber kappas[j]."""
    xyz, tri = _mesh(xyz, tri)
    n = tri.shape[0]
    rowptr, col = near_pairs(xyz, tri, eta)
    k = np.ascontiguousarray(np.atleast_1d(np.asarray(kappas, dtype=np.complex128)))
    dT = np.zeros((k.size, col.size), dtype=np.complex128)
    if col.size:
        _check(lib().or_nearfield_correction(_d(xyz), xyz.shape[0], tri.ctypes.data_as(_i32p), n,
                                             rowptr.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p),
                                             k.view(np.float64).ctypes.data_as(_dp), k.size, float(rtol),
                                             dT.view(np.float64).ctypes.data_as(_dp)))
    return rowptr, col, dT
