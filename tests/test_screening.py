"""The near-field screening and exponential polynomials (csrc/screening.h) against mpmath.

The P2P kernels evaluate C(x) = erfc(x) + (2/sqrt(pi)) x e^{-x^2} as
e^{-x^2} (erfcx(x) + 2x/sqrt(pi)) with erfcx from a polynomial in a Moebius-transformed
variable.  These tests re-evaluate the polynomials in FP64 the way the kernels do and bound the
absolute error of C, and the relative error of the reduced-cost exponential, on the whole range.
"""
import math
import os
import re

import mpmath as mp
import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2606_19059_amd", "csrc", "screening.h")


def _consts():
    src = open(HDR).read()
    scal = {k: float(v) for k, v in re.findall(r"constexpr double (k\w+) = ([^;{]+);", src)}
    arrs = {k: [float(v) for v in body.split(",")]
            for k, body in re.findall(r"constexpr double (k\w+)\[\d+\] = \{([^}]*)\};", src)}
    return scal, arrs


def _c_ref(x):
    mp.mp.dps = 30
    return np.array([float(mp.erfc(v) + 2 * v * mp.exp(-v * v) / mp.sqrt(mp.pi)) for v in map(mp.mpf, x)])


def _eval_u(x, c, K, A, B):
    """FP32 form: polynomial in u = A t + B, t = (x - K)/(x + K)."""
    t = (x - K) / (x + K)
    u = A * t + B
    q = np.full_like(x, c[-1])
    for a in c[-2::-1]:
        q = q * u + a
    return np.exp(-x * x) * (q + 2.0 * x / math.sqrt(math.pi))


def _eval_t(x, m, lead, K):
    """FP64 form: t = 1 - 2K/(x + K), monic Horner from t + m[deg-1], plus g x with
    g = (2/sqrt(pi))/lead, times lead."""
    t = 1.0 - (2.0 * K) * (1.0 / (x + K))
    q = t + m[-1]
    for a in m[-2::-1]:
        q = q * t + a
    return np.exp(-x * x) * (lead * ((2.0 / math.sqrt(math.pi) / lead) * x + q))


def test_screening_polynomials_meet_their_bounds():
    s, arrs = _consts()
    K, A, B, X = s["kScreenK"], s["kScreenA"], s["kScreenB"], s["kScreenXmax"]
    x = np.linspace(0.0, X, 2601)
    ref = _c_ref(x)
    for tag, bound in (("64", 5e-15), ("64s", 5e-12), ("64f", 3e-10)):
        err = np.max(np.abs(_eval_t(x, arrs["kScreenM" + tag], s["kScreenLead" + tag], K) - ref))
        assert err < bound, (tag, err)
    e32 = np.max(np.abs(_eval_u(x, arrs["kScreenC32"], K, A, B) - ref))
    assert e32 < 2e-9, e32


def test_screening_representations_agree():
    """The monic t-basis (FP64) and the u-basis (FP32) come from one Chebyshev interpolant: at
    the FP32 degree's neighbours the two forms differ only by the truncation, so a wrong
    substitution u = A t + B or a wrong leading coefficient shows up as a large difference."""
    s, arrs = _consts()
    K, A, B, X = s["kScreenK"], s["kScreenA"], s["kScreenB"], s["kScreenXmax"]
    x = np.linspace(0.0, X, 801)
    d = np.max(np.abs(_eval_t(x, arrs["kScreenM64s"], s["kScreenLead64s"], K) - _eval_u(x, arrs["kScreenC32"], K, A, B)))
    assert d < 2e-9, d


def test_exponential_polynomials_meet_their_bounds():
    """The reduced-cost exponentials: e^{-y} = 2^z, z = -y log2(e) = n + s, n = rint(z),
    2^s = lead p(s) with p the monic degree-8 (level 1) or degree-7 (level 2) polynomial of
    screening.h, evaluated by Horner in FP64 as the kernels do; relative error against mpmath
    over the P2P range 0 <= y < 42.3."""
    s, arrs = _consts()
    y = np.linspace(0.0, 42.3, 20001)
    z = -y * (1.0 / math.log(2.0))
    n = np.rint(z)
    f = z - n
    assert np.all(np.abs(f) <= 0.5)
    mp.mp.dps = 30
    ref = np.array([float(mp.exp(-mp.mpf(v))) for v in y])
    for tag, bound in (("1", 2e-12), ("2", 7e-11)):
        m = arrs["kExpM" + tag]
        p = f + m[-1]
        for a in m[-2::-1]:
            p = p * f + a
        err = np.max(np.abs(np.ldexp(s["kExpLead" + tag] * p, n.astype(int)) / ref - 1.0))
        assert err < bound, (tag, err)
