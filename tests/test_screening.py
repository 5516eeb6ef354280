"""The near-field screening polynomial (csrc/screening.h) against mpmath.

The P2P kernels evaluate C(x) = erfc(x) + (2/sqrt(pi)) x e^{-x^2} as
e^{-x^2} (erfcx(x) + 2x/sqrt(pi)) with erfcx from a polynomial in a Moebius-transformed
variable.  This test re-evaluates that polynomial in FP64 exactly as the kernels do and
bounds the absolute error of C on the whole fitted range.
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
    scal = dict(re.findall(r"constexpr double (kScreen[A-Za-z]+) = ([^;]+);", src))
    arrs = {k: [float(v) for v in body.split(",")]
            for k, body in re.findall(r"constexpr double (kScreenC\w+)\[\d+\] = \{([^}]*)\};", src)}
    return {k: float(v) for k, v in scal.items()}, arrs


def _eval(x, c, K, A, B):
    t = (x - K) / (x + K)
    u = A * t + B
    q = np.full_like(x, c[-1])
    for a in c[-2::-1]:
        q = q * u + a
    return np.exp(-x * x) * (q + 2.0 * x / math.sqrt(math.pi))


def test_screening_polynomials_meet_their_bounds():
    s, arrs = _consts()
    K, A, B, X = s["kScreenK"], s["kScreenA"], s["kScreenB"], s["kScreenXmax"]
    mp.mp.dps = 30
    x = np.linspace(0.0, X, 2601)
    ref = np.array([float(mp.erfc(v) + 2 * v * mp.exp(-v * v) / mp.sqrt(mp.pi)) for v in map(mp.mpf, x)])
    e64 = np.max(np.abs(_eval(x, arrs["kScreenC64"], K, A, B) - ref))
    e64s = np.max(np.abs(_eval(x, arrs["kScreenC64s"], K, A, B) - ref))
    e32 = np.max(np.abs(_eval(x, arrs["kScreenC32"], K, A, B) - ref))
    e64f = np.max(np.abs(_eval(x, arrs["kScreenC64f"], K, A, B) - ref))
    assert e64 < 5e-15, e64
    assert e64s < 5e-12, e64s
    assert e32 < 2e-9, e32
    assert e64f < 3e-10, e64f


def test_exponential_polynomials_meet_their_bounds():
    """The reduced-cost exponentials: e^{-y} = 2^n p(f), n = rint(-y log2 e), f = -y - n ln 2
    (|f| <= ln2/2), with p the degree-8 (level 1) or degree-7 (level 2) polynomial of
    screening.h, evaluated by Horner in FP64 as the kernels do; relative error against mpmath
    over the P2P range 0 <= y < 42.3."""
    src = open(HDR).read()
    polys = {k: [float(v) for v in body.split(",")]
             for k, body in re.findall(r"constexpr double (kExpC\w+)\[\d+\] = \{([^}]*)\};", src)}
    y = np.linspace(0.0, 42.3, 20001)
    n = np.rint(-y / math.log(2))
    f = -y - n * math.log(2)
    mp.mp.dps = 30
    ref = np.array([float(mp.exp(-mp.mpf(v))) for v in y])
    for name, bound in (("kExpC1", 2e-12), ("kExpC2", 7e-11)):
        c = polys[name]
        p = np.full_like(f, c[-1])
        for a in c[-2::-1]:
            p = p * f + a
        err = np.max(np.abs(np.ldexp(p, n.astype(int)) / ref - 1.0))
        assert err < bound, (name, err)
