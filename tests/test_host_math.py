"""Host checks of the library's own transcendental and Bessel arithmetic (CPU only).

* devmath.h's branch-free sincos_cw and exp_cw (Cody and Waite's reduction with economised
  series), compiled for the host by hipcc from the very header the kernels include, against
  long-double sinl, cosl and expl: sin and cos within 2 units of 2^-52 absolute (the header
  states 1.0-1.8), exp within 1 unit of 2^-52 relative, over the range the sweep uses
  (|x| <= 40), the whole admissible range (|x| <= 1e6 resp. 708), small arguments and points
  within a few ulps of multiples of pi/2.
* The Chebyshev (Jacobi-Anger) generator's Bessel values: a transcription of its loop (Miller's
  backward recurrence from J_M = 2^-1000, eight steps per trip with the 2^-400 rescale, the
  block's values recorded on the way down, normalised by J_0 + 2 sum J_2k = 1) and of the
  host's choice of the start index M (10 above the truncation length of the tail bound, rounded
  up to a multiple of 8), against scipy.special.jv over the admissible x = beta r in
  (1e-7, beta diam], within 1.5e-15 absolute (the values are at most 1); and, for BF16 and
  FP16 entries, M at the truncation length itself, within 1e-8.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import jv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_03938_amd", "csrc")


@pytest.fixture(scope="module")
def devmath_report(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc is not available")
    exe = str(tmp_path_factory.mktemp("devmath") / "devmath_check")
    subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    "-o", exe, os.path.join(ROOT, "tests", "host", "devmath_check.cpp")], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.splitlines():
        f = line.split()
        rows[(f[0], f[1])] = [float(v) for v in f[3:]]
    return rows


def test_sincos_error_bound(devmath_report):
    for rng in ("kernel_range", "full_range", "small", "near_half_pi_multiples"):
        s_err, c_err = devmath_report[("sincos", rng)]
        print(rng, s_err, c_err)
        assert s_err <= 2.0 and c_err <= 2.0, rng


def test_exp_error_bound(devmath_report):
    for rng in ("kernel_range", "full_range"):
        (err,) = devmath_report[("exp", rng)]
        print(rng, err)
        assert err <= 1.0, rng


def _cheb_length(x, block, tol, lmax=96):
    """The host's rule: smallest L > x/2 with 2 (x/2)^L / L! / (1 - (x/2)^2/(L+1)) <= tol,
    rounded up to whole blocks; also the unrounded length."""
    term = 2.0
    for L in range(1, lmax):
        term *= 0.5 * x / L
        q = 0.25 * x * x / (L + 1)
        if L > 0.5 * x and q < 1.0 and term / (1.0 - q) <= tol:
            return min((L + block - 1) // block * block, lmax - 1), L
    return lmax, lmax


def _miller_block(x, M, L0, nops):
    """J_{L0} .. J_{L0+nops-1} at x as the generator's loop forms them."""
    tx = 2.0 / x
    jp, jc = 0.0, 2.0 ** -1000
    S, f = 2.0 * jc, 1.0

    def steps8(l, track, jp, jc, S, f):
        t = l * tx
        for i in range(1, 9):
            jn = t * jc - jp
            jp, jc = jc, jn
            t -= tx
            if i % 2 == 0:
                S += 2.0 * jc
        sc = 2.0 ** -400 if abs(jc) > 2.0 ** 400 else 1.0
        jp, jc, S = jp * sc, jc * sc, S * sc
        if track:
            f *= sc
        return jp, jc, S, f

    l = M
    while l > L0 + nops:
        jp, jc, S, f = steps8(l, False, jp, jc, S, f)
        l -= 8
    jb = [0.0] * nops
    t = (L0 + nops) * tx
    for j in range(nops - 1, -1, -1):
        jn = t * jc - jp
        jp, jc = jc, jn
        t -= tx
        jb[j] = jc
        if j % 2 == 0:
            S += 2.0 * jc
    l = L0
    while l > 0:
        jp, jc, S, f = steps8(l, True, jp, jc, S, f)
        l -= 8
    S -= jc
    return [v * f / S for v in jb]


@pytest.mark.parametrize("xmax,tol", [(3.0 * np.sqrt(2.0), 1e-14), (6.0, 1e-14), (12.0, 1e-14), (6.0, 1e-9),
                                      (6.0, 1e-5)])
def test_miller_recurrence_matches_scipy(xmax, tol):
    L, need = _cheb_length(xmax, 8, tol)
    M = max((need + 10 + 7) // 8 * 8, L)
    xs = np.concatenate([[1e-7, 1e-4, 1e-2], np.linspace(0.05, xmax, 300)])
    worst = 0.0
    for x in xs:
        for L0 in range(0, L, 8):
            got = _miller_block(float(x), M, L0, 8)
            ref = jv(np.arange(L0, L0 + 8), x)
            worst = max(worst, float(np.max(np.abs(np.array(got) - ref))))
    print(f"x <= {xmax:.3f}, L = {L}, M = {M}: max |J - jv| = {worst:.2e}")
    assert worst <= 1.5e-15


@pytest.mark.parametrize("xmax,tol", [(1.0, 1e-5), (3.0 * np.sqrt(2.0), 1e-5), (6.0, 1e-6), (12.0, 1e-5),
                                      (12.0, 1e-6), (30.0, 1e-6)])
def test_miller_recurrence_16bit_start(xmax, tol):
    """For BF16 and FP16 entries (truncation tolerances 1e-5 and 1e-6) the recurrence starts at
    the truncation length itself (no margin above it, rounded up to a multiple of 8): the
    Bessel values it forms stay within 1e-8 of scipy's, far below the 2^-9 / 2^-12 rounding of
    the entries."""
    L, need = _cheb_length(xmax, 8, tol)
    M = max((need + 7) // 8 * 8, L)
    xs = np.concatenate([[1e-7, 1e-4, 1e-2], np.linspace(0.05, xmax, 200)])
    worst = 0.0
    for x in xs:
        for L0 in range(0, L, 8):
            got = _miller_block(float(x), M, L0, 8)
            worst = max(worst, float(np.max(np.abs(np.array(got) - jv(np.arange(L0, L0 + 8), x)))))
    print(f"x <= {xmax:.3f}, tol {tol}: L = {L}, M = {M}: max |J - jv| = {worst:.2e}")
    assert worst <= 1e-8
