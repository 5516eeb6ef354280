"""Plans chosen by the cost model from the tolerance alone: accuracy and predicted time."""
import numpy as np
import pytest

import oracle
from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("box,tol,prec,n", [((1, 1, 1), 1e-6, "fp32", 200_000), ((1, 1, 2), 1e-8, "fp64", 50_000)])
def test_auto_plan_meets_tolerance_and_its_prediction(box, tol, prec, n):
    import paper_2606_19059_amd as E

    x, f = W.particles(n, box, seed=31)
    X, F = torch.from_numpy(x).cuda(), torch.from_numpy(f).cuda()
    pl = E.Plan(box, tol, precision=prec, n_max=n, timers=True)
    ws = pl.workspace(n)
    u = torch.empty_like(X)
    for _ in range(2):
        pl.eval(X, F, out=u, workspace=ws)
    torch.cuda.synchronize()
    ms = []
    for _ in range(3):
        pl.eval(X, F, out=u, workspace=ws)
        torch.cuda.synchronize()
        ms.append(pl.stage_ms()["total"])
    measured = float(np.median(ms))
    pred = pl.info["predicted_ms"]
    tgt = W.sample_targets(n, 12, seed=131)
    err = oracle.rel_err(u.cpu().numpy()[:, tgt], oracle.ewald_sum(x, f, box, targets=tgt))
    print("auto plan %s grid %s P %d: measured %.2f ms, predicted %.2f ms, sampled err %.2e"
          % (prec, pl.info["grid"], pl.info["P"], measured, pred, err))
    assert err <= tol
    assert pred / 3 < measured < 3 * pred
