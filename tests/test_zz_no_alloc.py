"""ewald_eval_noalloc (workspace in the library's built-in device array) against ewald_eval.

Called through the C ABI on two evaluations in a row, the second with fewer particles (the
array keeps the first call's contents), in the default and the deterministic mode, FP64 and
FP32 bulk.  Bars: bitwise equality in the deterministic mode (same kernels, same order);
1e-12 of the result's max in the default mode (the symmetric P2P adds with atomics, so two
runs agree to rounding only).  Sizes above the array are refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


@pytest.mark.parametrize("precision,tol,deterministic", [("fp64", 1e-8, True), ("fp64", 1e-6, False),
                                                         ("fp32", 1e-5, False), ("fp32", 1e-6, True)])
def test_noalloc_matches_eval_on_two_calls(precision, tol, deterministic):
    import paper_2606_19059_amd as E

    lib = E.load()
    box = (1.0, 1.0, 2.0)
    pl = E.Plan(box, tol, grid=(32, 32, 64), n_max=60000, precision=precision, deterministic=deterministic)
    for n, seed in ((60000, 71), (7000, 72)):
        assert pl.workspace_bytes(n) <= E.NOALLOC_MAX_WORKSPACE
        x, f = W.particles(n, box, seed=seed, dist="blobs" if seed == 72 else "uniform", n_blobs=3)
        X, F = _dev(x), _dev(f)
        ref = pl.eval(X, F)
        u = torch.full_like(X, float("nan"))
        s = torch.cuda.current_stream()
        rc = lib.ewald_eval_noalloc(pl.handle, n, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                    ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        assert rc == E.EWALD_OK, lib.ewald_last_error().decode()
        torch.cuda.synchronize()
        a, b = u.cpu().numpy(), ref.cpu().numpy()
        if deterministic:
            assert np.array_equal(a, b)
        else:
            assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_noalloc_refuses_sizes_above_its_array():
    import paper_2606_19059_amd as E

    pl = E.Plan((1.0, 1.0, 1.0), 1e-8, grid=(64, 64, 64), n_max=1_000_000)
    n = 1_000_000
    assert pl.workspace_bytes(n) > E.NOALLOC_MAX_WORKSPACE
    X = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(E.EwaldError) as ei:
        pl.eval_noalloc(X, X)
    assert ei.value.code == E.EWALD_ENOMEM
    assert "scratch" in str(ei.value)
    # the plan still evaluates a size that fits
    x, f = W.particles(20000, (1.0, 1.0, 1.0), seed=73)
    u = pl.eval_noalloc(_dev(x), _dev(f))
    ref = pl.eval(_dev(x), _dev(f))
    torch.cuda.synchronize()
    assert torch.max(torch.abs(u - ref)).item() <= 1e-12 * torch.max(torch.abs(ref)).item()
