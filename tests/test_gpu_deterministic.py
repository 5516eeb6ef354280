"""The deterministic mode (EWALD_FLAG_DETERMINISTIC) against the CPU oracle, and its
bitwise reproducibility.

The mode evaluates every ordered pair from the target's side (one-sided P2P, no atomics)
in four variants, chosen by the plan: the full-precision FP64 pair formula (tol < 1e-10),
the two reduced-cost FP64 formulas (1e-10 <= tol < 1e-8, tol >= 1e-8) and the FP32 formula
(FP32 bulk).  Each is compared element by element with the oracle's real-space sum
(eq. g-near) at the plan's xi and r_c, within the bound of its formula:
* full FP64: 1e-12 of the array's max (same sums, different summation order);
* reduced-cost FP64, 1e-10 <= tol < 1e-8: 1e-10 (|dC| < 4e-12, exponential < 1.1e-12);
* reduced-cost FP64, tol >= 1e-8: 1e-9 (|dC| < 3e-10, exponential < 5.6e-11);
* FP32 formula: 2e-6 (single-precision pair terms, FP64 accumulation).
Reproducibility needs a fixed order of the particles inside every grid cell; cells of more
than 16, 256 and thousands of particles take three different sorting kernels, so the
clustered case below fills cells of every class.
"""
import numpy as np
import pytest

import oracle
from oracle import spectral as S
from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (box, grid, xi, r_c, P, Gaussian shape m)
BOX, GRID, XI, RC, P, M = (1.0, 1.3, 0.8), (16, 32, 64), 9.0, 0.30, 12, 5.8

# (precision, tol, near-field bound): the FP64 pair formula's three accuracy levels and FP32 bulk
VARIANTS = [("fp64", 1e-11, 1e-12), ("fp64", 1e-9, 1e-10), ("fp64", 1e-6, 1e-9), ("fp32", 1e-5, 2e-6)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def plan(E, precision, tol, n, box=BOX, grid=GRID, xi=XI, rc=RC, deterministic=True):
    return E.Plan(box, tol, xi=xi, r_c=rc, grid=grid, P=P, window_shape=M, n_max=n, precision=precision,
                  deterministic=deterministic)


def clustered(n_uniform, cells, seed):
    """Uniform particles plus, for each (count, cell corner, cell edge) of `cells`, `count`
    particles drawn uniformly inside that grid cell."""
    rng = np.random.default_rng(seed)
    parts = [rng.random((3, n_uniform)) * np.array(BOX).reshape(3, 1)]
    for count, corner, edge in cells:
        parts.append(np.array(corner).reshape(3, 1) + rng.random((3, count)) * np.array(edge).reshape(3, 1))
    x = np.concatenate(parts, axis=1)
    f = rng.standard_normal(x.shape)
    f -= f.mean(axis=1, keepdims=True)
    return x, f


@pytest.mark.parametrize("precision,tol,bound", VARIANTS)
def test_deterministic_near_field_matches_oracle(precision, tol, bound):
    import paper_2606_19059_amd as E

    n = 2500
    x, f = W.particles(n, BOX, seed=41)
    pl = plan(E, precision, tol, n)
    assert pl.info["deterministic"]
    un, uf = pl.eval_parts(dev(x), dev(f))
    un = host(un)
    ref = oracle.real_space(x, f, BOX, XI, RC)
    err = maxrel(un, ref)
    print("%s tol %g: deterministic P2P max rel err %.2e (bound %g)" % (precision, tol, err, bound))
    assert err < bound
    # the far field is the same stages as in the default mode
    far_bound = 1e-11 if precision == "fp64" else 2e-5
    assert maxrel(host(uf), S.far_field(x, f, BOX, GRID, XI, P, M)) < far_bound


@pytest.mark.parametrize("precision,tol,bound", VARIANTS)
def test_deterministic_is_bitwise_reproducible_with_crowded_cells(precision, tol, bound):
    """Three evaluations agree bitwise although cells hold 1 to 3000 particles (the per-cell
    order comes from the three cell-sorting kernels, not from the scatter's atomics)."""
    import paper_2606_19059_amd as E

    h = [BOX[d] / GRID[d] for d in range(3)]
    cells = [(3000, (0.5, 0.65, 0.4), h),          # one cell with 3000 particles
             (200, (0.25, 0.3, 0.1), h),            # 200 in one cell
             (40, (0.75, 0.9, 0.7), h),              # 40 in one cell
             (600, (0.1, 0.1, 0.6), [3 * v for v in h])]  # ~22 per cell over 27 cells
    x, f = clustered(1500, cells, seed=43)
    n = x.shape[1]
    pl = plan(E, precision, tol, n)
    X, F = dev(x), dev(f)
    runs = [host(pl.eval(X, F)) for _ in range(3)]
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], runs[2])
    un, _ = pl.eval_parts(X, F)
    err = maxrel(host(un), oracle.real_space(x, f, BOX, XI, RC))
    print("%s crowded cells: P2P max rel err %.2e" % (precision, err))
    assert err < bound
    # the default (symmetric, atomic) mode agrees to its rounding
    s = host(plan(E, precision, tol, n, deterministic=False).eval(X, F))
    scale = np.max(np.abs(runs[0]))
    assert np.max(np.abs(s - runs[0])) < (1e-12 if precision == "fp64" and tol < 1e-10 else 2 * bound) * scale


def test_spread_grid_is_bitwise_reproducible_with_crowded_cells():
    """P2G sums each grid point in the sorted order, so the grid is bitwise reproducible too
    (in both modes: the sort is shared)."""
    import paper_2606_19059_amd as E

    h = [BOX[d] / GRID[d] for d in range(3)]
    x, f = clustered(800, [(5000, (0.3, 0.3, 0.3), h), (100, (0.6, 0.6, 0.2), h)], seed=44)
    pl = plan(E, "fp64", 1e-11, x.shape[1], deterministic=False)
    X, F = dev(x), dev(f)
    g1, g2 = host(pl.spread(X, F)), host(pl.spread(X, F))
    assert np.array_equal(g1, g2)
    assert maxrel(g1, S.p2g(x, f, BOX, GRID, P, M)) < 1e-12
