"""The oracle's pins must be sensitive: each plausible mistake planted into a copy of the
oracle's C source (compiled on the CPU into a temporary library) makes at least one pin
fail.  The shipped oracle is never modified."""
import ctypes
import os
import subprocess
import tempfile
from math import factorial

import numpy as np
import pytest

import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bem_oracle.c")
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _build(mutation):
    src = open(SRC).read()
    old, new = mutation
    assert src.count(old) >= 1, old
    src = src.replace(old, new)
    d = tempfile.mkdtemp(prefix="oracle_mutant_")
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"],
                   check=True)
    L = ctypes.CDLL(so)
    L.or_apply_rows.argtypes = [_dp, ctypes.c_int64, _i32p, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, _i64p, ctypes.c_int64, _dp,
                                ctypes.c_int64, ctypes.c_int64, _dp]
    L.or_self_term_tri.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
    L.or_radon7.argtypes = [_dp, _dp]
    return L


def _row_sum_error(L, level, kappa, amplitude=0.0):
    xyz, tri = (synth.perturbed_icosphere(level, amplitude, seed=11) if amplitude
                else synth.icosphere(level))
    n = len(tri)
    rows = np.arange(0, n, max(1, n // 32)).astype(np.int64)
    V = np.ones((n, 1), dtype=np.complex128)
    Y = np.zeros((rows.size, 1), dtype=np.complex128)
    rc = L.or_apply_rows(xyz.ctypes.data_as(_dp), xyz.shape[0], tri.ctypes.data_as(_i32p), n,
                         kappa.real, kappa.imag, 0, rows.ctypes.data_as(_i64p), rows.size,
                         V.view(np.float64).ctypes.data_as(_dp), 1, 1,
                         Y.view(np.float64).ctypes.data_as(_dp))
    assert rc == 0
    lam0 = np.sin(kappa) * np.exp(1j * kappa) / kappa
    return np.abs(Y[:, 0] - lam0).max() / abs(lam0)


def _pins_pass(L):
    """A condensed version of the oracle pins; returns False as soon as one fails."""
    # quadrature: degree-5 exactness
    b = np.zeros(21)
    w = np.zeros(7)
    L.or_radon7(b.ctypes.data_as(_dp), w.ctypes.data_as(_dp))
    pts = b.reshape(7, 3) @ np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    for i in range(6):
        for j in range(6 - i):
            ex = factorial(i) * factorial(j) / factorial(i + j + 2)
            if abs(0.5 * np.sum(w * pts[:, 0] ** i * pts[:, 1] ** j) - ex) > 1e-14:
                return False
    # self term: equilateral closed form at k = 0
    s = 0.37
    P = np.array([0, 0, 0, s, 0, 0, s / 2, s * np.sqrt(3) / 2, 0], dtype=float)
    out = np.zeros(2)
    L.or_self_term_tri(P.ctypes.data_as(_dp), 0.0, 0.0, 0, out.ctypes.data_as(_dp))
    if abs(out[0] - np.sqrt(3) * s * np.arcsinh(np.sqrt(3)) / (4 * np.pi)) > 1e-15 or abs(out[1]) > 1e-15:
        return False
    # operator: row sums approach the sphere eigenvalue, also on an uneven mesh
    for amp in (0.0, 0.15):
        e3 = _row_sum_error(L, 3, 3.7 + 0.2j, amp)
        e4 = _row_sum_error(L, 4, 3.7 + 0.2j, amp)
        if not (e4 < 1e-2 and e3 / e4 > 3.0):
            return False
    return True


MUTANTS = {
    "exponent sign": ("cexp(I * k * r)", "cexp(-I * k * r)"),
    "missing 4 pi": ("/ (4.0 * PI * r)", "/ (PI * r)"),
    "target-row area weight": ("s += g->qw[7 * b + q] * kern;", "s += g->qw[7 * a + q] * kern;"),
    "swapped orbit weights": ("const double w1 = (155.0 + s) / 1200.0, w2 = (155.0 - s) / 1200.0;",
                              "const double w1 = (155.0 - s) / 1200.0, w2 = (155.0 + s) / 1200.0;"),
    "self-term radius": ("radial(k, dist / cos(phi), d)", "radial(k, dist * cos(phi), d)"),
    "collocation at a vertex": ("const double *x = g->cen + 3 * a;", "const double *x = g->vtx + 9 * a;"),
    "dropped quadrature point": ("for (int q = 0; q < 7; ++q) {\n        const double *y",
                                 "for (int q = 1; q < 7; ++q) {\n        const double *y"),
}


def test_unmutated_copy_passes():
    assert _pins_pass(_build(("/* ------------------------------------------------------------------- entries --- */",
                              "/* entries */")))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    assert not _pins_pass(_build(MUTANTS[name])), name
