"""The step kernel's FP64 exp, log, log1p, sin/cos(pi x), reciprocal and
square root (paper_2203_11043_amd/csrc/gccd_fp64.h), built for the host from
the same source (only fma, frexp, ldexp, rint and IEEE comparison; the
reciprocal and square root start from a single-precision estimate where the
device takes its hardware one, then the same Newton steps), against 40-digit
references: at most 2 units in the last place over the
arguments the time step gives them (Eq. (2): ln |E|^2, the exponent of
(|E|/Ec)^beta, log1p of it; Box-Muller: ln u, the angles 2 u of
u = (w + 1/2) 2^-32 and sqrt(-2 ln u); Eq. (3): sqrt(2 D dt)) and over the
functions' whole ranges (the reciprocal and square root over single
precision's normal range, where the host estimate exists), plus the special
values.  The forms without special-case tests that the step takes (exp_fin,
log1p_fin) equal the full ones bit for bit in their ranges."""
import os
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "helpers", "fp64_check.cpp")
INC = os.path.join(ROOT, "paper_2203_11043_amd", "csrc")


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    d = tmp_path_factory.mktemp("fp64")
    exe = str(d / "fp64_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", INC, SRC, "-o", exe,
                    "-lm"], check=True)

    def call(xe, xl, xp, xs, xr=None):
        n = len(xe)
        if xr is None:
            xr = np.ones(n)
        inp = np.concatenate([xe, xl, xp, xs, xr]).astype(np.float64)
        fi, fo = str(d / "in.bin"), str(d / "out.bin")
        inp.tofile(fi)
        subprocess.run([exe, fi, fo, str(n)], check=True)
        out = np.fromfile(fo, dtype=np.float64).reshape(9, n)
        return out
    return call


def args(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.float64)
    u = (w + 0.5) * 2.0**-32
    xe = np.concatenate([rng.uniform(-30.0, 30.0, n // 2),            # Eq. (2) exponents
                         rng.uniform(-745.0, 709.0, n - n // 2)])     # whole range
    xl = np.concatenate([u[: n // 3],                                 # Box-Muller ln u
                         10.0 ** rng.uniform(-2.0, 14.0, n // 3),     # |E|^2 in (V/cm)^2
                         2.0 ** rng.uniform(-1070.0, 1023.0, n - 2 * (n // 3))])
    xp = 10.0 ** rng.uniform(-20.0, 6.0, n)                           # (|E|/Ec)^beta
    xs = np.concatenate([2.0 * u[: n // 2], rng.uniform(-8.0, 8.0, n - n // 2)])
    xr = np.concatenate([-2.0 * np.log(u[: n // 3]),                  # Box-Muller radius^2
                         10.0 ** rng.uniform(-14.0, -6.0, n // 3),    # 2 D dt in cm^2
                         10.0 ** rng.uniform(-37.0, 38.0, n - 2 * (n // 3))])
    return xe, xl, xp, xs, xr


def ulp_error(got, ref):
    """|got - ref| in units of the spacing of doubles at ref."""
    ref = mp.mpf(ref)
    if ref == 0:
        return 0.0 if got == 0 else float("inf")
    e = int(mp.floor(mp.log(abs(ref), 2)))
    ulp = mp.mpf(2) ** (max(e, -1022) - 52)
    return float(abs(mp.mpf(got) - ref) / ulp)


def test_against_40_digit_references(run):
    mp.mp.dps = 40
    n = 6000
    xe, xl, xp, xs, xr = args(n, 5)
    out = run(xe, xl, xp, xs, xr)
    worst = {}
    for name, xs_, refs, k, bound in (
            ("exp", xe, lambda x: mp.exp(x), 0, 2.0),
            ("log", xl, lambda x: mp.log(x), 1, 2.0),
            ("log1p", xp, lambda x: mp.log1p(x), 2, 2.0),
            ("sinpi", xs, lambda x: mp.sinpi(x), 3, 2.0),
            ("cospi", xs, lambda x: mp.cospi(x), 4, 2.0),
            ("recip", xr, lambda x: 1 / x, 5, 1.0),
            ("sqrt", xr, lambda x: mp.sqrt(x), 6, 1.0),
            ("exp_fin", xe, lambda x: mp.exp(x), 7, 2.0),
            ("log1p_fin", xp, lambda x: mp.log1p(x), 8, 2.0)):
        errs = [ulp_error(out[k][i], refs(mp.mpf(float(xs_[i])))) for i in range(n)]
        worst[name] = max(errs)
        print(f"[fp64] {name}: max {worst[name]:.2f} ulp over {n} arguments", flush=True)
        assert worst[name] <= bound, name


def test_special_values(run):
    inf, nan = float("inf"), float("nan")
    xe = np.array([0.0, -0.0, 1.0, -1.0, inf, -inf, nan, 709.7, -745.1, 800.0, -800.0, 1e-300])
    xl = np.array([1.0, 0.0, -0.0, inf, nan, -1.0, 2.0, 0.5, 5e-324, 1.7976931348623157e308,
                   0.7071067811865476, 1.4142135623730951])
    xp = np.array([0.0, 1e-300, 1e-17, inf, nan, 1.0, -0.5, 1e300, 2.0**-53, 2.0**-52, 3.0, 1e6])
    xs = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, -0.5, 4.0, 1e-20])
    xr = np.array([1.0, 4.0, 2.0, 0.25, 1.7, 2.414213562373095, 3.0, 1e-30, 1e30, 2.0**-126,
                   2.0**126, 1.0 - 2.0**-53])
    out = run(xe, xl, xp, xs, xr)
    e, l, p, s, c, rc, sq, ef, pf = out
    assert e[0] == 1.0 and e[1] == 1.0 and e[4] == inf and e[5] == 0.0 and np.isnan(e[6])
    assert e[9] == inf and e[10] == 0.0 and e[11] == 1.0
    assert np.isfinite(e[7]) and e[8] > 0.0
    assert l[0] == 0.0 and l[1] == -inf and l[2] == -inf and l[3] == inf and np.isnan(l[4])
    assert np.isnan(l[5]) and l[6] == np.log(2.0) and l[7] == -np.log(2.0)
    assert abs(l[8] - np.log(5e-324)) <= 1e-12 and abs(l[9] - np.log(1.7976931348623157e308)) < 1e-12
    assert p[0] == 0.0 and p[1] == 1e-300 and p[2] == 1e-17 and p[3] == inf and np.isnan(p[4])
    assert abs(p[5] - np.log(2.0)) <= 2e-16 and abs(p[6] - np.log(0.5)) <= 2e-16
    # exact quadrant values
    assert list(s[:9]) == [0.0, s[1], 1.0, s[3], 0.0, s[5], -1.0, s[7], 0.0]
    assert list(c[[0, 2, 4, 6, 8]]) == [1.0, 0.0, -1.0, 0.0, 1.0]
    assert abs(s[1] - np.sqrt(0.5)) <= 2e-16 and abs(c[1] - np.sqrt(0.5)) <= 2e-16
    assert s[9] == -1.0 and s[10] == 0.0 and c[10] == 1.0 and s[11] == np.pi * 1e-20
    # exact squares and powers of two give exact results
    assert list(rc[[0, 1, 2, 3]]) == [1.0, 0.25, 0.5, 4.0] and rc[9] == 2.0**126
    assert list(sq[[0, 1, 3]]) == [1.0, 2.0, 0.5] and sq[9] == 2.0**-63 and sq[10] == 2.0**63
    assert abs(sq[2] - np.sqrt(2.0)) <= 2.3e-16 and abs(sq[6] - np.sqrt(3.0)) <= 2.3e-16
    # the forms without special cases agree with the full ones in their ranges
    # (exp_fin on [-745.2, 709.8], log1p_fin on finite y > -1, where 1 + y
    # rounding to 1 gives y itself)
    fin = (xe >= -745.2) & (xe <= 709.8)
    assert np.array_equal(ef[fin], e[fin])
    fin = np.isfinite(xp) & (xp > -1.0)
    assert np.array_equal(pf[fin], p[fin])


def test_coefficients_are_the_fitted_ones():
    """The polynomial coefficients in gccd_fp64.h are the ones
    fp64_coefficients.py fits (40-digit Chebyshev fits rounded to double),
    each within its printed accuracy."""
    import re
    import sys
    script = os.path.join(INC, "fp64_coefficients.py")
    out = subprocess.run([sys.executable, script], capture_output=True, text=True,
                         check=True).stdout
    fitted = [float(v) for v in re.findall(r"^\s+(-?[0-9.e+-]+),$", out, flags=re.M)]
    assert len(fitted) == 12 + 7 + 7 + 8
    header = open(os.path.join(INC, "gccd_fp64.h")).read()
    for line in out.splitlines():
        if "max relative error" in line:
            assert float(line.split()[-1]) < 5e-16, line
    for v in fitted:
        if v != 1.0:  # the leading terms, written as 1.0 among others
            assert repr(v) in header, v
