"""The pair-count diagnostic (ewald_count_pairs) against a brute-force count.

The count is what the P2P roofline is priced on (flops per ordered pair inside r_c), so it
is pinned here by its plain definition: every ordered pair (i, j), i != j, and every
periodic image p with 0 < |x_i - x_j + p| < r_c, enumerated in numpy over all images that
can fall inside r_c.  Integer result: compared exactly.
"""
import math

import numpy as np
import pytest

from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def brute_pairs(x, box, rc):
    L = np.asarray(box, dtype=np.float64)
    k = [int(math.ceil(rc / L[d])) for d in range(3)]  # |d + m L| < r_c needs |m| <= ceil(r_c / L)
    total = 0
    for a in range(0, x.shape[1], 512):
        d = x[:, a:a + 512, None] - x[:, None, :]
        for m0 in range(-k[0], k[0] + 1):
            for m1 in range(-k[1], k[1] + 1):
                for m2 in range(-k[2], k[2] + 1):
                    r2 = ((d[0] + m0 * L[0]) ** 2 + (d[1] + m1 * L[1]) ** 2 + (d[2] + m2 * L[2]) ** 2)
                    total += int(np.count_nonzero((r2 < rc * rc) & (r2 > 0.0)))
    return total


CASES = [
    # box, grid, xi, r_c, n, distribution
    ((1.0, 1.0, 1.0), (32, 32, 32), 11.44, 0.387, 2000, "uniform"),  # r_c > L/3: two cells per side
    ((1.0, 1.3, 0.8), (16, 32, 64), 9.0, 0.30, 1531, "uniform"),
    ((1.0, 1.0, 1.0), (8, 8, 8), 3.0, 0.45, 300, "uniform"),
    ((0.25, 0.25, 16.0), (8, 8, 512), 30.0, 0.1, 3000, "uniform"),
    ((1.0, 1.0, 1.0), (64, 64, 64), 20.0, 0.2, 1500, "blobs"),
]


@pytest.mark.parametrize("box,grid,xi,rc,n,dist", CASES)
def test_pair_count_matches_brute_force(box, grid, xi, rc, n, dist):
    import paper_2606_19059_amd as E

    x, f = W.particles(n, box, seed=61, dist=dist, n_blobs=7, sigma=0.02)
    x = np.concatenate([x, x[:, :5]], axis=1)  # five exact duplicates: r = 0, not counted
    f = np.concatenate([f, f[:, :5]], axis=1)
    pl = E.Plan(box, 1e-8, xi=xi, r_c=rc, grid=grid, P=8, n_max=x.shape[1])
    X = torch.from_numpy(x).to("cuda")
    F = torch.from_numpy(f).to("cuda")
    got = pl.count_pairs(X, F)
    want = brute_pairs(x, box, rc)
    print("box %s r_c %g n %d: %d pairs" % (box, rc, x.shape[1], got))
    assert got == want


def test_pair_count_of_nothing_is_zero():
    import paper_2606_19059_amd as E

    pl = E.Plan((1, 1, 1), 1e-6, grid=(32, 32, 32), n_max=10)
    z = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    assert pl.count_pairs(z, z) == 0
    one = torch.tensor([[0.5], [0.5], [0.5]], dtype=torch.float64, device="cuda")
    assert pl.count_pairs(one, one) == 0
