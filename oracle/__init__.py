"""FP64 CPU oracle for the triply periodic Stokeslet sum -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2606_19059_amd``) and never imports it.

Two references live here:

* :func:`ewald_sum` -- the plain definition.  A classical Ewald sum (real-space
  image sum with ``erfc`` + direct Fourier sum over the reciprocal lattice +
  self term), written in C (``ewald_oracle.c``), accurate to ~1e-13 relative.
  It follows Sec. 2 (eq. potentials, g-near, GFk) with the 3-periodic lattice.
* :mod:`oracle.spectral` -- the spectral Ewald steps of Algorithm "se"
  (P2P, P2G, FFT, CNV, IFFT, G2P, SUM) in the paper's order, with the Gaussian
  window, in numpy FP64.  It gives the same discrete quantities as the fast
  method (grid values, far field), so it pins each fast stage element by
  element; it is itself pinned against :func:`ewald_sum`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libewald_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc + OpenMP (a second or two)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        lib.ewo_real_space.argtypes = [i64, dp, dp, i64, ip, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.ewo_recip.argtypes = [i64, dp, dp, i64, ip, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.ewo_direct_sphere.argtypes = [i64, dp, dp, dp, ctypes.c_double, dp]
        lib.ewo_real_space_st.argtypes = [i64, dp, dp, i64, ip, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.ewo_recip_st.argtypes = [i64, dp, dp, i64, ip, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.ewo_num_threads.restype = ctypes.c_int
        lib.ewo_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().ewo_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the following oracle calls (for timing on fewer cores)."""
    _load().ewo_set_num_threads(int(n))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(x, f, L):
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    assert x.ndim == 2 and x.shape[0] == 3 and f.shape == x.shape
    return x, f, L


def _targets(targets):
    if targets is None:
        return None, None
    t = np.ascontiguousarray(targets, dtype=np.int64)
    return t, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def wrap(x, L):
    """Positions wrapped into [0, L) per component (periodic box)."""
    L = np.asarray(L, dtype=np.float64).reshape(3, 1)
    y = x - L * np.floor(x / L)
    y = np.where(y >= L, y - L, y)
    return np.where(y < 0.0, 0.0, y)


def real_space(x, f, L, xi, r_cut, targets=None):
    """Near-field sum of eq. (g-near) over all images with 0 < |r| < r_cut.

    Returns (3, n_targets).  With ``r_cut`` equal to the fast method's cutoff
    this is exactly what the P2P step computes (up to rounding).
    """
    lib = _load()
    x, f, L = _prep(x, f, L)
    n = x.shape[1]
    t, tp = _targets(targets)
    nt = n if t is None else t.shape[0]
    u = np.zeros((3, nt), dtype=np.float64)
    if n == 0 or nt == 0:
        return u
    lib.ewo_real_space(n, _dptr(x), _dptr(f), nt, tp, _dptr(L), float(xi), float(r_cut), _dptr(u))
    return u


def recip_space(x, f, L, xi, k_max, targets=None):
    """Fourier-space sum of eq. (GFk) over k != 0, |k| <= k_max.  Returns (3, n_targets)."""
    lib = _load()
    x, f, L = _prep(x, f, L)
    n = x.shape[1]
    t, tp = _targets(targets)
    nt = n if t is None else t.shape[0]
    u = np.zeros((3, nt), dtype=np.float64)
    if n == 0 or nt == 0:
        return u
    lib.ewo_recip(n, _dptr(x), _dptr(f), nt, tp, _dptr(L), float(xi), float(k_max), _dptr(u))
    return u


def self_term(f, xi, targets=None):
    """-G^F(0) f_i = -(4 xi / sqrt(pi)) f_i: removes the i = j, p = 0 term the smooth far field includes."""
    f = np.asarray(f, dtype=np.float64)
    if targets is not None:
        f = f[:, np.asarray(targets)]
    return -(4.0 * xi / math.sqrt(math.pi)) * f


def direct_sphere(x, f, L, R):
    """Brute-force image sum of G over whole image cells with |p| <= R (no splitting)."""
    lib = _load()
    x, f, L = _prep(x, f, L)
    u = np.zeros_like(x)
    lib.ewo_direct_sphere(x.shape[1], _dptr(x), _dptr(f), _dptr(L), float(R), _dptr(u))
    return u


def stresslet_tensor(q, nrm):
    """S_j = q_j n_j^T as 9 rows: S[3 b + c, j] = q_bj n_cj."""
    q = np.asarray(q, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    return np.ascontiguousarray(np.einsum("bj,cj->bcj", q, nrm).reshape(9, -1))


def real_space_st(x, S, L, xi, r_cut, targets=None):
    """Near-field stresslet sum (screened T^N over all images with 0 < |r| < r_cut) for the
    source tensors S (9, n).  Returns (3, n_targets)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    n = x.shape[1]
    assert S.shape == (9, n)
    t, tp = _targets(targets)
    nt = n if t is None else t.shape[0]
    u = np.zeros((3, nt), dtype=np.float64)
    if n == 0 or nt == 0:
        return u
    lib.ewo_real_space_st(n, _dptr(x), _dptr(S), nt, tp, _dptr(L), float(xi), float(r_cut), _dptr(u))
    return u


def recip_space_st(x, S, L, xi, k_max, targets=None):
    """Fourier-space stresslet sum over k != 0, |k| <= k_max.  Returns (3, n_targets)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    n = x.shape[1]
    t, tp = _targets(targets)
    nt = n if t is None else t.shape[0]
    u = np.zeros((3, nt), dtype=np.float64)
    if n == 0 or nt == 0:
        return u
    lib.ewo_recip_st(n, _dptr(x), _dptr(S), nt, tp, _dptr(L), float(xi), float(k_max), _dptr(u))
    return u


def default_xi(L, n, n_targets=None):
    """Oracle's own split parameter: real-space radius r_o = 6/xi_o.

    Full evaluation: r_o = min(L)/2 (only the nearest image can fall inside).
    Sampled targets with many sources: r_o = min(L), which keeps the number of
    reciprocal vectors (and so the structure-factor cost, O(n K)) small.
    """
    Lmin = float(np.min(L))
    if n_targets is not None and n_targets * 50 < n:
        return 6.0 / Lmin
    return 12.0 / Lmin


def ewald_sum(x, f, L, targets=None, xi=None, parts=False, q=None, nrm=None):
    """The periodic Stokeslet sum by classical Ewald summation, FP64, ~1e-13 accurate.

    xi_o is the oracle's own split parameter (the result does not depend on it);
    r_cut = 6/xi_o and k_max = 12 xi_o put both truncations below 1e-15.  With ``q`` and
    ``nrm`` (3, n) the stresslet sources q n^T of the combined single and double layer sum
    (Sec. 2.3) are added.  Returns (3, n_targets), or (total, real, recip, self) when ``parts``.
    """
    x, f, L = _prep(x, f, L)
    n = x.shape[1]
    nt = n if targets is None else len(targets)
    if xi is None:
        xi = default_xi(L, n, None if targets is None else nt)
    r_cut = 6.0 / xi
    k_max = 12.0 * xi
    ur = real_space(x, f, L, xi, r_cut, targets)
    uk = recip_space(x, f, L, xi, k_max, targets)
    us = self_term(f, xi, targets)
    if q is not None:
        S = stresslet_tensor(q, nrm)
        ur = ur + real_space_st(x, S, L, xi, r_cut, targets)
        uk = uk + recip_space_st(x, S, L, xi, k_max, targets)
    tot = ur + uk + us
    if parts:
        return tot, ur, uk, us
    return tot


def rel_err(u, ref):
    """Relative RMS error ||u - ref||_2 / ||ref||_2 over all targets and components."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(u - ref) / (den if den > 0 else 1.0))


def max_rel_err(u, ref):
    """max_i |u_i - ref_i| / max_i |ref_i| (maximum-norm relative error)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(u - ref)) / (den if den > 0 else 1.0))
