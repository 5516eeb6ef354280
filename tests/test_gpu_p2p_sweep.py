"""Near-field (P2P) and far-field (P2G, FFT, G2P) parity over a seeded sweep of sizes, boxes,
grids, splitting parameters and particle distributions, against the oracle's classical
real-space sum and spectral far field (element by element).

The sizes straddle the 64-target chunks (1, 63, 64, 65, 2047, 2049 ...); the distributions put
many particles in one tile (dense batches: the balanced drain's queue and extra rounds),
leave most tiles empty, or repeat positions.  FP64 plans use the full-precision pair formula
(tol < 1e-10): 1e-12 of the array's max; the same FP64 cases at tol 1e-9 and 1e-7 run the
reduced-cost formulas (1e-10 and 1e-9 of the max); FP32-bulk plans: 2e-6 (FP32 pair terms
accumulated in FP64).  Stresslet sources are checked on a subset the same way."""
import numpy as np
import pytest

import oracle
from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _E():
    import paper_2606_19059_amd as E

    E.load()
    return E


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def positions(kind, n, box, rng):
    L = np.asarray(box, float)[:, None]
    if kind == "uniform":
        return rng.random((3, n)) * L
    if kind == "dense":  # most particles in a small ball: a few very full tiles
        c = rng.random((3, 1)) * L
        x = c + 0.02 * float(min(box)) * rng.standard_normal((3, n))
        return np.mod(x, L)
    if kind == "sparse":  # a few clusters far apart: most tiles empty
        c = rng.random((3, 3)) * L
        x = c[:, rng.integers(0, 3, n)] + 0.05 * float(min(box)) * rng.standard_normal((3, n))
        return np.mod(x, L)
    if kind == "repeats":  # every position taken twice (exact duplicates)
        h = rng.random((3, (n + 1) // 2)) * L
        return np.concatenate([h, h], axis=1)[:, :n]
    raise ValueError(kind)


# (n, box, grid, xi, r_c, distribution, precision)
SWEEP = [
    (1, (1.0, 1.0, 1.0), (16, 16, 16), 6.0, 0.4, "uniform", "fp64"),
    (63, (1.0, 1.0, 1.0), (16, 16, 16), 6.0, 0.4, "uniform", "fp64"),
    (64, (1.0, 1.3, 0.8), (16, 32, 16), 8.0, 0.35, "uniform", "fp64"),
    (65, (1.0, 1.0, 2.0), (16, 16, 32), 7.0, 0.45, "uniform", "fp64"),
    (500, (1.0, 1.0, 1.0), (32, 32, 32), 10.0, 0.3, "dense", "fp64"),
    (777, (0.7, 1.3, 1.1), (16, 32, 32), 9.0, 0.3, "sparse", "fp64"),
    (1024, (1.0, 1.0, 1.0), (32, 32, 32), 11.0, 0.38, "repeats", "fp64"),
    (2047, (1.0, 1.0, 4.0), (16, 16, 64), 6.0, 0.5, "uniform", "fp64"),
    (2049, (1.0, 1.0, 1.0), (64, 64, 64), 14.0, 0.25, "dense", "fp64"),
    (3000, (1.0, 1.0, 1.0), (8, 8, 8), 3.0, 0.45, "uniform", "fp64"),
    (1531, (1.0, 1.3, 0.8), (16, 32, 64), 9.0, 0.3, "uniform", "fp32"),
    (2500, (1.0, 1.0, 1.0), (32, 32, 32), 10.0, 0.3, "dense", "fp32"),
]


@pytest.mark.parametrize("case", range(len(SWEEP)))
def test_p2p_sweep_matches_oracle(case):
    E = _E()
    n, box, grid, xi, rc, kind, prec = SWEEP[case]
    rng = np.random.default_rng(100 + case)
    x = positions(kind, n, box, rng)
    f = W.mean_free_forces(rng, n) if n > 1 else rng.standard_normal((3, n))
    tol = 1e-11 if prec == "fp64" else 1e-5
    pl = E.Plan(box, tol, xi=xi, r_c=rc, grid=grid, P=8, n_max=n, precision=prec)
    un, _ = pl.eval_parts(dev(x), dev(f))
    ref = oracle.real_space(x, f, box, xi, rc)
    err = maxrel(host(un), ref) if np.max(np.abs(ref)) > 0 else float(np.max(np.abs(host(un))))
    bound = 1e-12 if prec == "fp64" else 2e-6
    print("P2P sweep %d: n %d %s %s %s: max rel err %.2e" % (case, n, kind, prec, grid, err))
    assert err < bound


# the reduced-cost FP64 pair formulas (accuracy levels 1 and 2, chosen from the plan's tol), with
# the bound each level's formula error allows: level 1 (1e-10 <= tol < 1e-8) 1e-10, level 2 1e-9
LEVELS = [(1e-9, 1e-10), (1e-7, 1e-9)]


@pytest.mark.parametrize("case", [c for c in range(len(SWEEP)) if SWEEP[c][6] == "fp64"])
@pytest.mark.parametrize("level", range(len(LEVELS)))
def test_p2p_sweep_reduced_levels_match_oracle(case, level):
    E = _E()
    n, box, grid, xi, rc, kind, prec = SWEEP[case]
    tol, bound = LEVELS[level]
    rng = np.random.default_rng(400 + case)
    x = positions(kind, n, box, rng)
    f = W.mean_free_forces(rng, n) if n > 1 else rng.standard_normal((3, n))
    pl = E.Plan(box, tol, xi=xi, r_c=rc, grid=grid, P=8, n_max=n, precision=prec)
    un, _ = pl.eval_parts(dev(x), dev(f))
    ref = oracle.real_space(x, f, box, xi, rc)
    err = maxrel(host(un), ref) if np.max(np.abs(ref)) > 0 else float(np.max(np.abs(host(un))))
    print("P2P sweep %d at tol %g: n %d %s %s: max rel err %.2e" % (case, tol, n, kind, grid, err))
    assert err < bound


@pytest.mark.parametrize("case", [2, 4, 6, 8, 10])
def test_p2p_sweep_stresslet_matches_oracle(case):
    E = _E()
    n, box, grid, xi, rc, kind, prec = SWEEP[case]
    rng = np.random.default_rng(200 + case)
    x = positions(kind, n, box, rng)
    f = W.mean_free_forces(rng, n)
    q, nr = rng.standard_normal((3, n)), rng.standard_normal((3, n))
    tol = 1e-11 if prec == "fp64" else 1e-5
    pl = E.Plan(box, tol, xi=xi, r_c=rc, grid=grid, P=8, n_max=n, precision=prec, stresslet=True)
    un, _ = pl.eval_combined_parts(dev(x), dev(f), dev(q), dev(nr))
    ref = oracle.real_space(x, f, box, xi, rc) + oracle.real_space_st(x, oracle.stresslet_tensor(q, nr), box, xi, rc)
    err = maxrel(host(un), ref)
    bound = 1e-12 if prec == "fp64" else 2e-6
    print("P2P stresslet sweep %d: n %d %s %s: max rel err %.2e" % (case, n, kind, prec, err))
    assert err < bound


@pytest.mark.parametrize("case", [1, 3, 5, 8, 10, 11])
def test_far_field_sweep_matches_oracle(case):
    """G2P (16-target groups contracted on the matrix cores) and P2G on the same sweep, against
    the spectral oracle's far field."""
    from oracle import spectral as S

    E = _E()
    n, box, grid, xi, rc, kind, prec = SWEEP[case]
    rng = np.random.default_rng(300 + case)
    x = positions(kind, n, box, rng)
    f = W.mean_free_forces(rng, n)
    P = 8
    m = 0.94 * np.sqrt(np.pi * P)
    tol = 1e-11 if prec == "fp64" else 1e-5
    pl = E.Plan(box, tol, xi=xi, r_c=rc, grid=grid, P=P, window_shape=m, n_max=n, precision=prec)
    _, uf = pl.eval_parts(dev(x), dev(f))
    err = maxrel(host(uf), S.far_field(x, f, box, grid, xi, P, m))
    bound = 1e-11 if prec == "fp64" else 2e-5
    print("far-field sweep %d: n %d %s %s %s: max rel err %.2e" % (case, n, kind, prec, grid, err))
    assert err < bound
