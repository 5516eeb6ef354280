"""Host-side checks of the C ABI (no GPU): symbols, validation, parameter selection."""
import math
import os
import re

import pytest

import paper_2606_19059_amd as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ewald.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ewald_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = E.load()
    names = _declared()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(E.EXPORTS) == names
    assert "gfx950" in E.version()


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        E.load(str(tmp_path / "nope.so"))


@pytest.mark.parametrize(
    "kw, msg",
    [
        (dict(box=(0.0, 1, 1), tol=1e-6), "box"),
        (dict(box=(1, 1, 1), tol=0.5), "tol"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(32, 30, 32)), "grid"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(4, 32, 32)), "grid"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(32, 32, 32), P=7), "P"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(32, 32, 32), P=18), "P"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(32, 32, 32), r_c=1.5), "r_c"),
        (dict(box=(1, 1, 1), tol=1e-6, grid=(32, 32, 32), r_c=0.01), "r_c"),
        (dict(box=(1, 1, 1), tol=1e-6, n_max=-1), "n_max"),
    ],
)
def test_invalid_parameters_rejected(kw, msg):
    with pytest.raises(E.EwaldError, match=msg) as ei:
        E.resolve(**kw)
    assert ei.value.code == E.EWALD_EINVAL


def _EN(xi, rc):  # eq. (ese), near-field term
    return math.sqrt(112 / 9 * xi**4 * rc**3) * math.exp(-(xi * rc) ** 2)


def _EF(xi, h):  # eq. (ese), Fourier term
    return 4 / (3 * h) * math.sqrt(3.5) * math.exp(-math.pi**2 / (2 * h * xi) ** 2)


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8, 1e-10])
def test_parameters_follow_error_split(tol):
    """xi and r_c put E^N and E^F at tol/3 (Sec. 2.4 split), window error <= tol/3."""
    i = E.resolve((1, 1, 1), tol, grid=(64, 64, 64))
    h = 1.0 / 64
    assert _EF(i["xi"], h) == pytest.approx(tol / 3, rel=1e-6)
    assert _EN(i["xi"], i["r_c"]) == pytest.approx(tol / 3, rel=1e-6)
    assert i["err_window"] <= tol / 3 or i["P"] == 16
    assert i["P"] % 2 == 0 and 4 <= i["P"] <= 16
    B = i["tile"]
    assert B & (B - 1) == 0 and 2 <= B <= 16
    assert all(s * B * h >= i["r_c"] for s in i["stencil"])


def test_window_support_grows_as_tolerance_tightens():
    Ps = [E.resolve((1, 1, 1), t, grid=(128, 128, 128))["P"] for t in (1e-3, 1e-5, 1e-7, 1e-9)]
    assert Ps == sorted(Ps) and Ps[0] < Ps[-1]


def test_auto_grid_and_workspace():
    a = E.resolve((1, 1, 2), 1e-6, n_max=200_000)
    M = a["grid"]
    assert all(m & (m - 1) == 0 for m in M) and M[2] >= M[0]
    assert _EF(a["xi"], max(1 / M[0], 1 / M[1], 2 / M[2])) <= 1e-6 / 3 * (1 + 1e-6)
    b = E.resolve((1, 1, 2), 1e-6, n_max=400_000, grid=M, xi=a["xi"], r_c=a["r_c"], P=a["P"])
    assert b["workspace_bytes"] > a["workspace_bytes"]


def test_explicit_parameters_are_kept():
    i = E.resolve((1, 1, 1), 1e-6, xi=9.0, r_c=0.3, grid=(32, 32, 32), P=10, window_shape=5.1)
    assert (i["xi"], i["r_c"], i["grid"], i["P"], i["window_shape"]) == (9.0, 0.3, (32, 32, 32), 10, 5.1)


def test_fourier_stage_precision_follows_tolerance():
    """FP32 bulk keeps the grid and its transforms in FP32 down to tol 1e-6, FP64 below."""
    g = (64, 64, 64)
    assert not E.resolve((1, 1, 1), 1e-6, grid=g, precision="fp32")["fourier_fp64"]
    assert E.resolve((1, 1, 1), 1e-7, grid=g, precision="fp32")["fourier_fp64"]
    assert E.resolve((1, 1, 1), 1e-4, grid=g, precision="fp64")["fourier_fp64"]
    w32 = E.resolve((1, 1, 1), 1e-6, grid=g, precision="fp32", n_max=1000)["workspace_bytes"]
    w64 = E.resolve((1, 1, 1), 1e-7, grid=g, precision="fp32", n_max=1000)["workspace_bytes"]
    assert w64 - w32 >= 0.9 * 3 * 64 ** 3 * 4  # the FP64 grid (tile tables differ slightly)


@pytest.mark.parametrize("box,tol,prec,n", [((1, 1, 1), 1e-8, "fp64", 10**6), ((1, 1, 2), 1e-6, "fp32", 10**5),
                                            ((1, 1, 1), 1e-4, "fp32", 3000)])
def test_cost_model_picks_the_cheapest_resolvable_grid(box, tol, prec, n):
    """With only the tolerance given, the plan is the grid of least predicted time among the
    power-of-two grids (each resolved by the error split), and keeps the split."""
    i = E.resolve(box, tol, precision=prec, n_max=n)
    assert i["predicted_ms"] > 0
    assert i["err_near"] <= tol / 3 * 1.0001 and i["err_far"] <= tol / 3 * 1.0001
    m0 = min(i["grid"])
    for m in (m0 // 2, m0 * 2):
        if m < 8 or m * max(box) / min(box) > 512:
            continue
        g = tuple(int(m * b / min(box)) for b in box)
        try:
            j = E.resolve(box, tol, precision=prec, n_max=n, grid=g)
        except E.EwaldError:
            continue
        assert j["predicted_ms"] >= i["predicted_ms"] * (1 - 1e-9), (g, j["predicted_ms"], i["predicted_ms"])


def test_cost_model_grows_with_work():
    a = E.resolve((1, 1, 1), 1e-6, precision="fp32", n_max=10**5, grid=(128, 128, 128))
    b = E.resolve((1, 1, 1), 1e-6, precision="fp32", n_max=10**6, grid=(128, 128, 128))
    c = E.resolve((1, 1, 1), 1e-8, precision="fp64", n_max=10**6, grid=(128, 128, 128))
    assert a["predicted_ms"] < b["predicted_ms"] < c["predicted_ms"]


def test_stresslet_plans():
    """EWALD_FLAG_STRESSLET sizes a larger workspace (sorted tensors, 9-component grid) and is
    refused together with EWALD_FLAG_DETERMINISTIC."""
    g = (32, 32, 32)
    a = E.resolve((1, 1, 1), 1e-6, grid=g, n_max=1000)
    b = E.resolve((1, 1, 1), 1e-6, grid=g, n_max=1000, stresslet=True)
    assert b["stresslet"] and not a["stresslet"]
    assert b["workspace_bytes"] >= a["workspace_bytes"] + 6 * 32**3 * 8 + 48 * 1000
    with pytest.raises(E.EwaldError) as ei:
        E.resolve((1, 1, 1), 1e-6, grid=g, n_max=1000, stresslet=True, deterministic=True)
    assert ei.value.code == E.EWALD_EUNSUPPORTED


@pytest.mark.parametrize("precision,tol,grid,elem", [("fp64", 1e-8, (32, 32, 64), 8), ("fp32", 1e-5, (64, 64, 128), 4),
                                                     ("fp32", 1e-7, (32, 32, 64), 8)])
def test_info_self_coefficient_and_grid_bytes(precision, tol, grid, elem):
    """The plan reports the self-term coefficient (equal to the oracle's self term per unit
    force) and the byte size of the diagnostic grids (element type by fourier_fp64)."""
    import numpy as np

    import oracle

    info = E.resolve((1.0, 1.0, 2.0), tol, precision=precision, grid=grid, n_max=1000)
    f = np.ones((3, 1))
    assert info["self_coef"] == pytest.approx(-oracle.self_term(f, info["xi"])[0, 0], rel=1e-15)
    assert info["fourier_fp64"] == (elem == 8)
    assert info["grid_bytes"] == 3 * grid[0] * grid[1] * grid[2] * elem
