"""Spectral Ewald steps in the paper's order, numpy FP64 -- TEST INFRASTRUCTURE.

Algorithm "se" (Sec. 2.2): P2P, P2G, FFT, CNV, IFFT, G2P, SUM, here on the
3-periodic box with the Gaussian window.  Plain and slow: dense index
arithmetic, ``np.add.at`` for the spreading sum, ``numpy.fft`` for the
transforms.  It computes the same discrete quantities as the fast method, so
it pins each fast stage element by element, and is itself pinned against the
classical Ewald sum of :mod:`oracle` (see the tests).

Conventions (each a reading of the paper, recorded in the design notes):

* grid points g_l = l h, l = 0..M-1 per dimension, h = L/M;
* the P-point stencil of a point y: anchor a = floor(y/h) - (P/2 - 1), points
  a..a+P-1 (mod M); P even (Sec. 3.2, anchor rule);
* Gaussian window, per dimension w0(d) = exp(-alpha d^2) for |d| < P h / 2,
  alpha = 2 m^2 / (P h)^2 with shape parameter m (the classic Gaussian window
  the paper cites in Sec. 2.2); its Fourier transform is taken untruncated,
  w0^(k) = sqrt(pi/alpha) exp(-k^2 / (4 alpha));
* or the truncated Kaiser-Bessel window of Sec. 2.2 (``window="kb"``):
  w0(d) = I0(beta sqrt(1 - d^2/a^2)) / I0(beta) for |d| < a, a = P h / 2,
  beta = m P (m = 2.5 when not given, the paper's choice), with the closed-form
  transform of the truncated window (the KB transform pair),
  w0^(k) = 2a sinh(sqrt(beta^2 - (k a)^2)) / (sqrt(beta^2 - (k a)^2) I0(beta))
  (sin and sqrt((k a)^2 - beta^2) when k a > beta);
* P2G without h^3 (eq. p2g), G2P with h^3 (eq. g2p), forward DFT unnormalised,
  inverse DFT with 1/prod(M) (numpy's convention), eq. (sca) in between;
* the k = 0 mode and the Nyquist planes (index M/2) are set to zero.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import i0 as _i0

from . import real_space, real_space_st, self_term, stresslet_tensor, wrap


def window_1d(dist, h, P, m, window="gaussian"):
    """The 1D window w0 at distances ``dist`` (open support |dist| < P h / 2)."""
    a = P * h / 2
    inside = np.abs(dist) < a
    if window == "kb":
        beta = (m if m else 2.5) * P
        z = np.clip(1.0 - (dist / a) ** 2, 0.0, None)
        w = _i0(beta * np.sqrt(z)) / _i0(beta)
    else:
        alpha = 2.0 * m * m / (P * h) ** 2
        w = np.exp(-alpha * dist * dist)
    return np.where(inside, w, 0.0)


def stencil_1d(y, Ld, Md, P, m, window="gaussian"):
    """Grid indices (n, P) and window weights (n, P) of the P-point stencil along one axis."""
    h = Ld / Md
    c = np.floor(y / h)
    t = y / h - c
    j = np.arange(P, dtype=np.float64)
    idx = (c[:, None].astype(np.int64) - (P // 2 - 1) + np.arange(P, dtype=np.int64)[None, :]) % Md
    dist = (j[None, :] - (P / 2 - 1) - t[:, None]) * h  # g_l - y
    return idx, window_1d(dist, h, P, m, window)


def window_hat_1d(k, Ld, Md, P, m, window="gaussian"):
    """Fourier transform of the 1D window at wave numbers k (Gaussian: untruncated)."""
    h = Ld / Md
    if window == "kb":
        a = P * h / 2
        beta = (m if m else 2.5) * P
        q = beta * beta - (k * a) ** 2
        sq = np.sqrt(np.abs(q))
        with np.errstate(invalid="ignore", divide="ignore"):
            hyp = np.where(q > 0, np.sinh(sq) / np.where(sq > 0, sq, 1.0), np.sin(sq) / np.where(sq > 0, sq, 1.0))
        hyp = np.where(sq == 0, 1.0, hyp)
        return 2.0 * a * hyp / _i0(beta)
    alpha = 2.0 * m * m / (P * h) ** 2
    return math.sqrt(math.pi / alpha) * np.exp(-k * k / (4.0 * alpha))


def p2g(x, f, L, M, P, m, chunk=4096, window="gaussian"):
    """eq. (p2g): phi(g_l) = sum_j w(g_l - y_j + p) f_j.  Returns (3, M1, M2, M3)."""
    x = wrap(np.asarray(x, dtype=np.float64), L)
    f = np.asarray(f, dtype=np.float64)
    M = [int(v) for v in M]
    phi = np.zeros((3, M[0] * M[1] * M[2]), dtype=np.float64)
    n = x.shape[1]
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i0, w0 = stencil_1d(x[0, s:e], L[0], M[0], P, m, window)
        i1, w1 = stencil_1d(x[1, s:e], L[1], M[1], P, m, window)
        i2, w2 = stencil_1d(x[2, s:e], L[2], M[2], P, m, window)
        flat = (i0[:, :, None, None] * M[1] + i1[:, None, :, None]) * M[2] + i2[:, None, None, :]
        w = w0[:, :, None, None] * w1[:, None, :, None] * w2[:, None, None, :]
        flat = flat.reshape(-1)
        for d in range(3):
            np.add.at(phi[d], flat, (w * f[d, s:e, None, None, None]).reshape(-1))
    return phi.reshape(3, M[0], M[1], M[2])


def wave_numbers(L, M):
    """Signed integer frequencies and wave vectors k_d = 2 pi n_d / L_d on the FFT index grid."""
    ns = [np.fft.fftfreq(int(M[d])) * int(M[d]) for d in range(3)]
    ks = [2.0 * math.pi * ns[d] / L[d] for d in range(3)]
    return ns, ks


def cnv(phihat, L, M, xi, P, m, window="gaussian"):
    """eq. (sca): vhat(k) = Ghat^F(k) / what(k)^2 phihat(k), Ghat^F from eq. (GFk).

    ``phihat``: (3, M1, M2, M3) complex, the unnormalised DFT of the grid.
    Zeroes k = 0 and the Nyquist planes.
    """
    ns, ks = wave_numbers(L, M)
    k0 = ks[0][:, None, None]
    k1 = ks[1][None, :, None]
    k2 = ks[2][None, None, :]
    kk = k0 * k0 + k1 * k1 + k2 * k2
    with np.errstate(divide="ignore", invalid="ignore"):
        g = 8.0 * math.pi / (kk * kk) * (1.0 + kk / (4.0 * xi * xi)) * np.exp(-kk / (4.0 * xi * xi))
    what = (
        window_hat_1d(ks[0], L[0], M[0], P, m, window)[:, None, None]
        * window_hat_1d(ks[1], L[1], M[1], P, m, window)[None, :, None]
        * window_hat_1d(ks[2], L[2], M[2], P, m, window)[None, None, :]
    )
    scale = g / (what * what)
    bad = kk == 0.0
    for d in range(3):
        nyq = np.zeros(int(M[d]), dtype=bool)
        nyq[int(M[d]) // 2] = True
        shape = [1, 1, 1]
        shape[d] = int(M[d])
        bad = bad | nyq.reshape(shape)
    scale = np.where(bad, 0.0, scale)
    kdot = k0 * phihat[0] + k1 * phihat[1] + k2 * phihat[2]
    return np.stack(
        [
            scale * (kk * phihat[0] - k0 * kdot),
            scale * (kk * phihat[1] - k1 * kdot),
            scale * (kk * phihat[2] - k2 * kdot),
        ]
    )


def cnv_stresslet(shat, L, M, xi, P, m, window="gaussian"):
    """The stresslet part of the combined CNV (Sec. 2.3, combined layers): 9 grid components in,
    3 out, vhat_a(k) = i A(k) / what(k)^2 P_abc(k) Shat_bc(k) with A = 8 pi / k^4 (1 + k^2/4 xi^2)
    e^{-k^2/4 xi^2} and P_abc = k^2 (delta_bc k_a + delta_ab k_c + delta_ac k_b) - 2 k_a k_b k_c.
    ``shat``: (9, M1, M2, M3) complex, row 3 b + c.  Zeroes k = 0 and the Nyquist planes."""
    ns, ks = wave_numbers(L, M)
    kv = [ks[0][:, None, None], ks[1][None, :, None], ks[2][None, None, :]]
    kk = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        A = 8.0 * math.pi / (kk * kk) * (1.0 + kk / (4.0 * xi * xi)) * np.exp(-kk / (4.0 * xi * xi))
    what = (
        window_hat_1d(ks[0], L[0], M[0], P, m, window)[:, None, None]
        * window_hat_1d(ks[1], L[1], M[1], P, m, window)[None, :, None]
        * window_hat_1d(ks[2], L[2], M[2], P, m, window)[None, None, :]
    )
    scale = A / (what * what)
    bad = kk == 0.0
    for d in range(3):
        nyq = np.zeros(int(M[d]), dtype=bool)
        nyq[int(M[d]) // 2] = True
        shape = [1, 1, 1]
        shape[d] = int(M[d])
        bad = bad | nyq.reshape(shape)
    scale = np.where(bad, 0.0, scale)
    out = []
    for a in range(3):
        w = 0.0
        for b in range(3):
            for c in range(3):
                Pabc = kk * ((b == c) * kv[a] + (a == b) * kv[c] + (a == c) * kv[b]) - 2.0 * kv[a] * kv[b] * kv[c]
                w = w + Pabc * shat[3 * b + c]
        out.append(1j * scale * w)
    return np.stack(out)


def g2p(v, x, L, M, P, m, chunk=4096, window="gaussian"):
    """eq. (g2p): u(x_i) = h1 h2 h3 sum_l w(x_i - g_l + p) v(g_l).  Returns (3, n)."""
    x = wrap(np.asarray(x, dtype=np.float64), L)
    M = [int(q) for q in M]
    h3 = (L[0] / M[0]) * (L[1] / M[1]) * (L[2] / M[2])
    vf = v.reshape(3, -1)
    n = x.shape[1]
    u = np.zeros((3, n), dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        i0, w0 = stencil_1d(x[0, s:e], L[0], M[0], P, m, window)
        i1, w1 = stencil_1d(x[1, s:e], L[1], M[1], P, m, window)
        i2, w2 = stencil_1d(x[2, s:e], L[2], M[2], P, m, window)
        flat = (i0[:, :, None, None] * M[1] + i1[:, None, :, None]) * M[2] + i2[:, None, None, :]
        w = w0[:, :, None, None] * w1[:, None, :, None] * w2[:, None, None, :]
        for d in range(3):
            u[d, s:e] = h3 * np.sum(w * vf[d][flat], axis=(1, 2, 3))
    return u


def far_grid(x, f, L, M, xi, P, m, window="gaussian"):
    """P2G -> FFT -> CNV -> IFFT: the real grid v(g_l) that G2P interpolates."""
    phi = p2g(x, f, L, M, P, m, window=window)
    phihat = np.fft.fftn(phi, axes=(1, 2, 3))
    vhat = cnv(phihat, L, M, xi, P, m, window)
    return np.real(np.fft.ifftn(vhat, axes=(1, 2, 3)))


def far_grid_combined(x, f, S, L, M, xi, P, m, window="gaussian"):
    """Combined single and double layer far grid: 3 + 9 components through P2G and the FFT,
    CNV maps them to 3, then the IFFT."""
    phi = p2g(x, f, L, M, P, m, window=window)
    sphi = np.concatenate([p2g(x, S[3 * r:3 * r + 3], L, M, P, m, window=window) for r in range(3)])
    vhat = cnv(np.fft.fftn(phi, axes=(1, 2, 3)), L, M, xi, P, m, window) + \
        cnv_stresslet(np.fft.fftn(sphi, axes=(1, 2, 3)), L, M, xi, P, m, window)
    return np.real(np.fft.ifftn(vhat, axes=(1, 2, 3)))


def far_field(x, f, L, M, xi, P, m, window="gaussian"):
    """u^F_h at every particle: G2P(IFFT(CNV(FFT(P2G(f))))).  Returns (3, n)."""
    v = far_grid(x, f, L, M, xi, P, m, window)
    return g2p(v, x, L, M, P, m, window=window)


def far_field_combined(x, f, S, L, M, xi, P, m, window="gaussian"):
    """u^F_h of the combined single and double layer sources at every particle."""
    return g2p(far_grid_combined(x, f, S, L, M, xi, P, m, window), x, L, M, P, m, window=window)


def spectral_ewald(x, f, L, M, xi, r_c, P, m, parts=False, window="gaussian", q=None, nrm=None):
    """Algorithm "se": u_h = u^N + u^F_h, plus the self term -(4 xi/sqrt(pi)) f (the stresslet
    part, with ``q`` and ``nrm``, needs none: T^F is odd).

    Returns (3, n), or (total, near, far, self) when ``parts``.
    """
    if q is not None:
        S = stresslet_tensor(q, nrm)
        un = real_space(x, f, L, xi, r_c) + real_space_st(x, S, L, xi, r_c)
        uf = far_field_combined(x, f, S, L, M, xi, P, m, window)
    else:
        un = real_space(x, f, L, xi, r_c)
        uf = far_field(x, f, L, M, xi, P, m, window)
    us = self_term(f, xi)
    tot = un + uf + us
    if parts:
        return tot, un, uf, us
    return tot
