"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test would fail for a plausible mistake somewhere in the oracle: a dropped
Ewald term, a wrong sign or factor in G^N or Ghat^F, a wrong self term, a wrong
reciprocal lattice, an index slip in the spectral stages.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import spectral as S
from paper_2606_19059_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- classical Ewald


@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.0, 1.0, 2.0), (0.7, 1.3, 1.1)])
def test_split_parameter_independence(box):
    """G^N + G^F = G, so the Ewald total cannot depend on xi (Sec. 2).

    A wrong relative factor between the real-space, Fourier and self terms, or a
    wrong exponent in either screening function, breaks this.
    """
    L = np.array(box)
    x, f = W.particles(7, L, seed=11)
    ref = oracle.ewald_sum(x, f, L, xi=6.0 / min(box))
    scale = np.max(np.abs(ref))
    for xi in (3.5 / min(box), 9.0 / min(box), 12.0 / min(box)):
        u = oracle.ewald_sum(x, f, L, xi=xi)
        # the self term 4 xi/sqrt(pi) |f| exceeds |u| several-fold: allow its rounding
        assert np.max(np.abs(u - ref)) / scale < 3e-12


def test_split_parameter_independence_with_net_force():
    """Also with sum f != 0 (the k = 0 mode is dropped on every side)."""
    L = np.array([1.0, 1.0, 1.0])
    rng = np.random.default_rng(5)
    x = rng.random((3, 5))
    f = rng.standard_normal((3, 5)) + 0.7
    a = oracle.ewald_sum(x, f, L, xi=5.0)
    b = oracle.ewald_sum(x, f, L, xi=10.0)
    assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-12


def test_hasimoto_single_stokeslet_constant():
    """N = 1 in a cube: u = -(4/3) K f / L with Hasimoto's lattice constant K."""
    g = json.load(open(os.path.join(GOLDEN, "hasimoto_cubic.json")))
    expected = -g["K"] * g["units_factor"]
    for Lside in (1.0, 2.5):
        L = np.array([Lside] * 3)
        x = np.array([[0.31], [0.17], [0.74]]) * Lside
        for fvec in ([1.0, 0.0, 0.0], [0.2, -0.5, 0.9]):
            f = np.array(fvec).reshape(3, 1)
            u = oracle.ewald_sum(x, f, L)
            assert np.allclose(u[:, 0], expected * f[:, 0] / Lside, rtol=1e-10, atol=1e-12)


def _surface_term(x, f, V):
    """Spherical-summation limit minus Ewald value, for zero net force.

    Derived from the k -> 0 behaviour of Ghat(k) S(k) e^{ik.x}: the O(1) term
    8 pi (I - kk) sum_j f_j [(k.x)(k.x_j) - (k.x_j)^2/2] (unit k) averaged over
    directions (<k_a k_b> = delta/3, <k_a k_b k_c k_d> = sym/15), divided by V.
    """
    n = x.shape[1]
    out = np.zeros_like(x)
    for i in range(n):
        xi_ = x[:, i]
        s = np.zeros(3)
        for j in range(n):
            xj, fj = x[:, j], f[:, j]
            s += (4 / 15) * fj * (xi_ @ xj) - (1 / 15) * (xi_ * (fj @ xj) + xj * (fj @ xi_))
            s += -(2 / 15) * fj * (xj @ xj) + (1 / 15) * xj * (fj @ xj)
        out[:, i] = 8 * math.pi / V * s
    return out


def test_brute_force_spherical_image_sums():
    """Plain image sums of G over growing spheres converge to the Ewald value.

    (i) after removing the best affine field c + A x_i the residual falls like R^-3;
    (ii) after removing the closed-form surface term the residual falls towards 0.
    """
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(9, L, seed=7)
    ue = oracle.ewald_sum(x, f, L)
    du = _surface_term(x, f, 1.0)
    X = np.hstack([np.ones((x.shape[1], 1)), x.T])
    fit_res, cf_res = [], []
    for R in (10.0, 20.0, 40.0):
        d = oracle.direct_sphere(x, f, L, R) - ue
        r = 0.0
        for c in range(3):
            coef, *_ = np.linalg.lstsq(X, d[c], rcond=None)
            r = max(r, float(np.max(np.abs(d[c] - X @ coef))))
        fit_res.append(r)
        cf_res.append(float(np.max(np.abs(d - du))))
    scale = np.max(np.abs(ue))
    assert fit_res[0] > fit_res[1] > fit_res[2]
    assert fit_res[2] / scale < 1e-6
    assert fit_res[0] / fit_res[1] > 5.0  # ~R^-3
    assert cf_res[0] > cf_res[2]
    assert cf_res[2] / scale < 1e-3
    # the surface term itself is O(1): without it the sums are far from the Ewald value
    assert np.max(np.abs(du)) / scale > 0.05


def test_mobility_matrix_symmetry():
    """G_per is even and symmetric: g . u(f) = f . u(g)."""
    L = np.array([1.0, 1.0, 2.0])
    rng = np.random.default_rng(3)
    x = rng.random((3, 12)) * L.reshape(3, 1)
    f = rng.standard_normal((3, 12))
    g = rng.standard_normal((3, 12))
    a = float(np.sum(g * oracle.ewald_sum(x, f, L)))
    b = float(np.sum(f * oracle.ewald_sum(x, g, L)))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_linearity_translation_permutation():
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(20, L, seed=9)
    _, g = W.particles(20, L, seed=10)
    u = oracle.ewald_sum(x, f, L)
    assert np.allclose(oracle.ewald_sum(x, 2.0 * f - 0.5 * g, L),
                       2.0 * u - 0.5 * oracle.ewald_sum(x, g, L), rtol=0, atol=1e-12 * np.max(np.abs(u)))
    assert np.all(oracle.ewald_sum(x, np.zeros_like(f), L) == 0.0)
    shift = np.array([[0.3], [-0.77], [1.6]])
    ut = oracle.ewald_sum(x + shift, f, L)
    assert np.max(np.abs(ut - u)) < 1e-12 * np.max(np.abs(u))
    p = np.random.default_rng(0).permutation(20)
    up = oracle.ewald_sum(x[:, p], f[:, p], L)
    assert np.max(np.abs(up - u[:, p])) < 1e-12 * np.max(np.abs(u))


def test_sampled_targets_match_full():
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(300, L, seed=12)
    u = oracle.ewald_sum(x, f, L)
    t = W.sample_targets(300, 17, seed=1)
    ut = oracle.ewald_sum(x, f, L, targets=t)
    assert np.max(np.abs(ut - u[:, t])) < 1e-12 * np.max(np.abs(u))


def test_real_space_reduces_to_stokeslet_for_tiny_xi():
    """As xi -> 0 the screened kernel G^N tends to the plain Stokeslet G (eq. g-near)."""
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(6, L, seed=2)
    rc = 0.45
    ur = oracle.real_space(x, f, L, 1e-7, rc)
    ref = np.zeros_like(ur)
    xw = oracle.wrap(x, L)
    for i in range(6):
        for j in range(6):
            for m in np.ndindex(3, 3, 3):
                r = xw[:, i] - xw[:, j] + (np.array(m) - 1.0)
                d = np.linalg.norm(r)
                if 0 < d < rc:
                    ref[:, i] += f[:, j] / d + r * (r @ f[:, j]) / d**3
    assert np.max(np.abs(ur - ref)) < 1e-6 * np.max(np.abs(ref))


def test_real_space_cutoff_saturates():
    """Beyond ~6/xi the real-space term no longer changes (erfc tail)."""
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(40, L, seed=4)
    a = oracle.real_space(x, f, L, 12.0, 0.5)
    b = oracle.real_space(x, f, L, 12.0, 0.8)
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(a))


# ---------------------------------------------------------------- spectral stages


def test_p2g_single_point_on_grid_node():
    """A unit force exactly on a grid node spreads the separable Gaussian e^{-beta j^2}."""
    L = (1.0, 1.0, 1.0)
    M = (16, 16, 16)
    P, m = 8, 4.5
    x = np.array([[5.0 / 16], [0.0], [9.0 / 16]])
    f = np.array([[1.0], [0.0], [0.0]])
    phi = S.p2g(x, f, L, M, P, m)
    beta = 2 * m * m / P**2
    offs = np.arange(-(P // 2 - 1), P // 2 + 1)
    w = np.exp(-beta * offs.astype(float) ** 2)
    # the node at offset +P/2 lies exactly at distance P h / 2: outside the open support
    w[offs == P // 2] = 0.0
    expect = np.zeros(M)
    for a, wa in zip(offs, w):
        for b, wb in zip(offs, w):
            for c, wc in zip(offs, w):
                expect[(5 + a) % 16, b % 16, (9 + c) % 16] = wa * wb * wc
    assert np.allclose(phi[0], expect, rtol=0, atol=1e-15)
    assert np.all(phi[1] == 0) and np.all(phi[2] == 0)


def test_p2g_translation_by_grid_cells_is_a_roll():
    L = (1.0, 1.0, 1.0)
    M = (12, 16, 8)
    x, f = W.particles(30, L, seed=21)
    phi = S.p2g(x, f, L, M, 6, 4.0)
    sh = np.array([[3.0 / 12], [-5.0 / 16], [1.0 / 8]])
    phi2 = S.p2g(x + sh, f, L, M, 6, 4.0)
    assert np.allclose(np.roll(phi, (3, -5, 1), axis=(1, 2, 3)), phi2, rtol=0, atol=1e-13)


def test_g2p_is_h3_times_p2g_transpose():
    """<g, G2P(v)> = h^3 <P2G(g), v>: interpolation is the adjoint of spreading (eq. p2g, g2p)."""
    L = (1.0, 1.2, 0.9)
    M = (10, 12, 8)
    x, g = W.particles(25, L, seed=31)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3,) + M)
    h3 = (L[0] / M[0]) * (L[1] / M[1]) * (L[2] / M[2])
    lhs = np.sum(g * S.g2p(v, x, L, M, 6, 4.2))
    rhs = h3 * np.sum(S.p2g(x, g, L, M, 6, 4.2) * v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_far_field_converges_to_fourier_sum():
    """P2G -> FFT -> CNV -> IFFT -> G2P approximates the direct Fourier sum (same xi).

    The error falls with the window support P and matches the window-error
    model within a small factor; a wrong deconvolution, Ghat^F factor or grid
    normalisation would leave an O(1) error.
    """
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(200, L, seed=1)
    xi = 11.444
    ref = oracle.recip_space(x, f, L, xi, 12 * 60)
    errs = []
    for P in (6, 8, 10):
        m = 0.94 * math.sqrt(math.pi * P)
        uf = S.far_field(x, f, L, (32, 32, 32), xi, P, m)
        errs.append(oracle.rel_err(uf, ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 6e-5 and errs[2] < 6e-6


def test_far_field_anisotropic_box():
    L = np.array([1.0, 1.0, 2.0])
    x, f = W.particles(150, L, seed=8)
    xi = 11.0
    ref = oracle.recip_space(x, f, L, xi, 12 * 60)
    uf = S.far_field(x, f, L, (32, 32, 64), xi, 10, 0.94 * math.sqrt(10 * math.pi))
    assert oracle.rel_err(uf, ref) < 6e-6


def test_spectral_total_matches_classical_ewald():
    """Algorithm se (P2P + far field + self) against the plain definition."""
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(400, L, seed=1)
    ue = oracle.ewald_sum(x, f, L)
    xi, rc = 10.282, 0.4798
    P = 12
    u = S.spectral_ewald(x, f, L, (32, 32, 32), xi, rc, P, 0.94 * math.sqrt(math.pi * P))
    assert oracle.rel_err(u, ue) < 3e-7


def test_kaiser_bessel_transform_matches_quadrature():
    """The closed-form transform of the truncated KB window (Sec. 2.2) against direct quadrature."""
    from scipy.integrate import quad

    h, P = 1.0 / 32, 8
    a = P * h / 2
    for k in (0.0, 17.0, 150.0, 2 * math.pi * 15):
        num, _ = quad(lambda d: float(S.window_1d(np.array([d]), h, P, 0, "kb")[0]) * math.cos(k * d), -a, a,
                      epsabs=1e-14, epsrel=1e-12, limit=400)
        ana = float(S.window_hat_1d(np.array([k]), 1.0, 32, P, 0, "kb")[0])
        assert abs(num - ana) < 1e-10 * abs(ana)


def test_kaiser_bessel_far_field_converges():
    L = np.array([1.0, 1.0, 1.0])
    x, f = W.particles(200, L, seed=1)
    xi = 11.444
    ref = oracle.recip_space(x, f, L, xi, 12 * 60)
    errs = [oracle.rel_err(S.far_field(x, f, L, (32, 32, 32), xi, P, 0, window="kb"), ref) for P in (4, 6, 8)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


# ---------------------------------------------------------------- stresslet (double layer) sources


def _stresslet_inputs(n, box, seed, orthogonal=False):
    rng = np.random.default_rng(seed)
    x = rng.random((3, n)) * np.asarray(box, dtype=float)[:, None]
    q = rng.standard_normal((3, n))
    nr = rng.standard_normal((3, n))
    if orthogonal:
        nr -= q * (np.sum(q * nr, 0) / np.sum(q * q, 0))
    return x, q, nr


@pytest.mark.parametrize("box", [(1.0, 1.0, 1.0), (1.0, 0.8, 1.7)])
def test_stresslet_sum_is_independent_of_xi(box):
    """The combined single and double layer sum does not depend on the split parameter: T^N
    and That^F (and G^N, Ghat^F) are two halves of one kernel only if they match."""
    x, q, nr = _stresslet_inputs(40, box, seed=21)
    f = np.random.default_rng(22).standard_normal((3, 40))
    lmin = min(box)
    us = [oracle.ewald_sum(x, f, box, xi=c / lmin, q=q, nrm=nr) for c in (5.0, 8.0, 12.0)]
    for u in us[1:]:
        assert oracle.max_rel_err(u, us[0]) < 1e-11


def test_stresslet_matches_finite_differences_of_stokeslets():
    """For q . n = 0, T_abc q_b n_c = (n.grad)(G q) + (q.grad)(G n) (T = d_c G_ab + d_b G_ac
    + 2 delta_bc d_a |r|^-1), so each stresslet equals the limit of four point forces +-q/eps
    at y -+ eps n/2 and +-n/eps at y -+ eps q/2.  Pins the stresslet oracle against the
    (independently pinned) Stokeslet oracle at spectator points; the error falls as eps^2."""
    box = (1.0, 1.0, 1.3)
    ns, nt = 12, 6
    ys, q, nr = _stresslet_inputs(ns, box, seed=7, orthogonal=True)
    xs = np.random.default_rng(8).random((3, nt)) * np.asarray(box)[:, None]
    x_all = np.concatenate([ys, xs], 1)
    z = np.zeros((3, nt))
    u_st = oracle.ewald_sum(x_all, np.zeros_like(x_all), box, q=np.concatenate([q, z], 1),
                            nrm=np.concatenate([nr, z], 1))[:, ns:]
    errs = []
    for eps in (1e-3, 1e-4):
        pos, frc = [], []
        for j in range(ns):
            for a, b in ((nr[:, j], q[:, j]), (q[:, j], nr[:, j])):
                pos += [ys[:, j] - 0.5 * eps * a, ys[:, j] + 0.5 * eps * a]
                frc += [b / eps, -b / eps]
        X = np.concatenate([np.array(pos).T, xs], 1)
        F = np.concatenate([np.array(frc).T, z], 1)
        errs.append(oracle.max_rel_err(oracle.ewald_sum(X, F, box)[:, 4 * ns:], u_st))
    assert errs[1] < 2e-6
    assert 50 < errs[0] / errs[1] < 200  # second order in eps


def test_stresslet_near_field_tends_to_the_bare_kernel():
    """As xi -> 0 the screened T^N tends to T = -6 r r r / r^5; checked against a direct image
    sum of T written out here."""
    box = (1.0, 1.0, 1.0)
    x, q, nr = _stresslet_inputs(7, box, seed=5)
    S = oracle.stresslet_tensor(q, nr)
    rc = 0.9
    un = oracle.real_space_st(x, S, box, 1e-7, rc)
    ref = np.zeros((3, 7))
    for i in range(7):
        for j in range(7):
            for m in np.ndindex(3, 3, 3):
                r = x[:, i] - x[:, j] + (np.array(m) - 1) * np.asarray(box)
                d = np.linalg.norm(r)
                if d == 0 or d >= rc:
                    continue
                Sj = S[:, j].reshape(3, 3)
                ref[:, i] += -6.0 * r * (r @ Sj @ r) / d**5
    assert oracle.max_rel_err(un, ref) < 1e-9


@pytest.mark.parametrize("window", ["gaussian", "kb"])
def test_spectral_combined_far_field_converges_to_direct_fourier_sum(window):
    """P2G of the 3 + 9 components, FFT, combined CNV (12 -> 3), IFFT, G2P converges to the
    classical Fourier sums of both kernels as the window support grows."""
    box = (1.0, 1.0, 1.0)
    x, q, nr = _stresslet_inputs(60, box, seed=3)
    f = np.random.default_rng(4).standard_normal((3, 60))
    St = oracle.stresslet_tensor(q, nr)
    xi = 8.0
    ref = oracle.recip_space_st(x, St, box, xi, 12 * xi) + oracle.recip_space(x, f, box, xi, 12 * xi)
    errs = []
    for P in (6, 10, 14):
        m = 0 if window == "kb" else 0.95 * math.sqrt(math.pi * P)
        errs.append(oracle.rel_err(S.far_field_combined(x, f, St, box, (32, 32, 32), xi, P, m,
                                                               window=window), ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < (1e-11 if window == "kb" else 1e-8)


# ---------------------------------------------------------------- error metrics


def test_rel_err_hand_computed():
    """Relative RMS error over all components: ||u - r||_2 / ||r||_2, by hand.

    r = [[3, 0], [0, 4]] has norm 5; u - r = [[0, 1], [-2, 2]] has norm 3, so 3/5.  A
    metric that averaged per component, used the max norm, or divided by ||u|| fails.
    """
    r = np.array([[3.0, 0.0], [0.0, 4.0]])
    u = np.array([[3.0, 1.0], [-2.0, 6.0]])
    assert oracle.rel_err(u, r) == pytest.approx(0.6, rel=1e-15)
    # symmetric in nothing: the reference's norm is the denominator
    assert oracle.rel_err(r, u) == pytest.approx(3.0 / math.sqrt(9 + 1 + 4 + 36), rel=1e-15)
    assert oracle.rel_err(r, r) == 0.0
    # zero reference: the absolute norm
    assert oracle.rel_err(np.array([[3.0], [4.0]]), np.zeros((2, 1))) == pytest.approx(5.0)


def test_max_rel_err_hand_computed():
    """max |u - r| / max |r| over all entries, by hand: max |u - r| = 2 (entry [1, 0]),
    max |r| = 4, so 0.5 (an RMS or per-entry relative metric gives another value)."""
    r = np.array([[3.0, 0.0], [-1.0, 4.0]])
    u = np.array([[3.5, 0.0], [1.0, 4.0]])
    assert oracle.max_rel_err(u, r) == pytest.approx(0.5, rel=1e-15)
    assert oracle.max_rel_err(r, r) == 0.0
    assert oracle.max_rel_err(np.array([[-7.0]]), np.zeros((1, 1))) == pytest.approx(7.0)
