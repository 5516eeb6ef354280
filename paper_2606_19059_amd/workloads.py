"""Seeded synthetic inputs (positions and forces) for every workload.

This module holds only random-number recipes; none of the Ewald method's
arithmetic.  Both the HIP path and the CPU oracle are fed from here.

The paper measures on synthetic particles only (uniform, normal and
sphere-surface distributions, Sec. 6 and appendix B); these recipes stand in
for them:

* generator ``numpy.random.default_rng(seed)`` (PCG64), positions drawn first,
  then forces;
* uniform: U[0, L_d) per component;
* blobs: ``n_blobs`` centres uniform in the box, equal shares of points per
  blob with N(0, sigma^2) offsets per component, wrapped periodically;
* forces: i.i.d. N(0, 1) per component, column mean subtracted (zero net force).

All arrays are (3, n) float64, component-major ("structure of arrays").
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def uniform_positions(rng, n, box):
    box = np.asarray(box, dtype=np.float64).reshape(3, 1)
    return rng.random((3, n)) * box


def blob_positions(rng, n, box, n_blobs, sigma):
    box = np.asarray(box, dtype=np.float64).reshape(3, 1)
    n_blobs = max(1, min(int(n_blobs), max(n, 1)))
    centres = rng.random((3, n_blobs)) * box
    owner = np.arange(n) % n_blobs
    x = centres[:, owner] + sigma * rng.standard_normal((3, n))
    x = x - box * np.floor(x / box)
    return np.where(x >= box, x - box, x)


def mean_free_forces(rng, n):
    f = rng.standard_normal((3, n))
    if n > 0:
        f -= f.mean(axis=1, keepdims=True)
    return f


def particles(n, box=(1.0, 1.0, 1.0), seed=0, dist="uniform", n_blobs=1000, sigma=None):
    """(x, f): seeded positions then mean-free N(0,1) forces, each (3, n) float64."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        x = uniform_positions(rng, n, box)
    elif dist == "blobs":
        s = 0.01 * float(min(box)) if sigma is None else sigma
        x = blob_positions(rng, n, box, n_blobs, s)
    else:
        raise ValueError("unknown distribution %r" % (dist,))
    f = mean_free_forces(rng, n)
    return x, f


def sample_targets(n, count, seed):
    """Seeded distinct target indices for sampled-oracle checks."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    box: tuple
    dist: str
    tol: float
    grid: tuple
    P: int
    precision: str
    seed: int
    n_blobs: int = 1000
    note: str = ""

    def make(self):
        return particles(self.n, self.box, self.seed, self.dist, self.n_blobs)


# The benchmark configurations (sizes, boxes, distributions, tolerances, grids
# and window supports of the spectral Ewald evaluation).  Seeds 1..5 by row,
# 11 for the 1e-6 headline case.
WORKLOADS = {
    "c1": Workload("c1", 1000, (1.0, 1.0, 1.0), "uniform", 1e-6, (32, 32, 32), 8, "fp64", 1,
                   note="small FP64 case, full oracle"),
    "c2": Workload("c2", 1_000_000, (1.0, 1.0, 1.0), "uniform", 1e-8, (128, 128, 128), 12, "fp64", 2,
                   note="FP64, 1e6 uniform, tol 1e-8"),
    "c3": Workload("c3", 10_000_000, (1.0, 1.0, 1.0), "blobs", 1e-5, (256, 256, 256), 8, "fp32", 3,
                   note="FP32 bulk, 1e7 in 1000 Gaussian blobs (sigma 0.01 L)"),
    "c4": Workload("c4", 4_000_000, (1.0, 1.0, 4.0), "uniform", 1e-7, (128, 128, 512), 10, "fp32", 4,
                   note="FP32 bulk + FP64 P2P accumulation, elongated box"),
    "H": Workload("H", 1_000_000, (1.0, 1.0, 1.0), "uniform", 1e-6, (128, 128, 128), 8, "fp32", 11,
                  note="1e-6 headline, FP32 bulk"),
}


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    box: tuple
    dist: str
    tol: float
    seed: int
    n_blobs: int = 1

    def make(self):
        return particles(self.n, self.box, self.seed, self.dist, self.n_blobs)


def serving_stream(n_requests, rate_per_s, seed=5, n_lo=1e3, n_hi=1e6, tols=(1e-4, 1e-6, 1e-8)):
    """Poisson arrivals of independent suspensions (the serving workload).

    N log-uniform in [n_lo, n_hi], cubic or 1x1x2 box, uniform or blob-clustered
    positions (max(1, N/1e4) blobs), tolerance drawn from ``tols``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = np.log10(n_lo), np.log10(n_hi)
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s) if rate_per_s > 0 else 0.0
        n = int(10 ** rng.uniform(lo, hi))
        box = (1.0, 1.0, 1.0) if rng.random() < 0.5 else (1.0, 1.0, 2.0)
        dist = "uniform" if rng.random() < 0.5 else "blobs"
        tol = float(tols[rng.integers(len(tols))])
        out.append(Request(i, t, n, box, dist, tol, int(1000 + i), max(1, n // 10_000)))
    return out
