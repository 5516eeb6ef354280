"""Serving: continuous admission of independent requests; each result equals its solo run."""
import numpy as np
import pytest

import oracle
from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _stream(n_req, seed):
    reqs = W.serving_stream(n_req, rate_per_s=2000.0, seed=seed, n_lo=1e3, n_hi=4e4)
    from paper_2606_19059_amd import serve

    return serve.make_jobs(reqs)


def _solo(job):
    from paper_2606_19059_amd import Plan, serve

    # a fresh plan with the server's parameters for this request (its size class)
    pl = Plan(job.box, job.tol, precision=serve.precision_for(job.tol), n_max=serve.Server.size_class(job.n))
    u = pl.eval(job.x.to("cuda"), job.f.to("cuda"))
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_results_equal_alone_and_in_the_mix():
    from paper_2606_19059_amd import serve

    jobs = _stream(30, seed=5)
    srv = serve.Server(n_slots=4)
    done = srv.run(jobs)
    torch.cuda.synchronize()
    assert len(done) == len(jobs)
    assert max(s.job is None for s in srv.slots)
    overlapped = sum(1 for a in done for b in done if a is not b and a.admitted < b.admitted < a.done)
    print("requests overlapping on the device: %d" % overlapped, serve.summarize(done))
    for j in done:
        mix = j.u.cpu().numpy()
        alone = _solo(j)
        d = np.max(np.abs(mix - alone)) / np.max(np.abs(alone))
        assert d <= 1e-12, (j.rid, j.n, j.tol, d)


def test_small_budget_forces_queueing_and_stays_correct():
    """A budget that fits the largest request only: in-flight bytes never exceed it, the
    largest request runs alone, smaller ones wait for memory, results stay correct."""
    from paper_2606_19059_amd import serve

    jobs = _stream(6, seed=9)
    for j in jobs:
        j.precision = serve.precision_for(j.tol)
    srv0 = serve.Server(n_slots=3)
    sizes = [srv0.footprint(j) for j in jobs]
    biggest = max(sizes)
    srv = serve.Server(n_slots=3, hbm_budget=biggest + 1024)
    done = srv.run(jobs)
    assert len(done) == 6
    assert srv.max_in_flight_bytes <= srv.budget
    big = max(done, key=lambda j: j.footprint)
    for b in done:
        if b is not big:
            assert not (big.admitted <= b.admitted < big.done or b.admitted <= big.admitted < b.done)
    assert srv.memory_waits > 0
    j = min(done, key=lambda j: j.n)
    ref = oracle.ewald_sum(j.x.numpy(), j.f.numpy(), j.box)
    assert oracle.rel_err(j.u.cpu().numpy(), ref) <= j.tol


def test_oversized_request_is_rejected():
    from paper_2606_19059_amd import serve

    jobs = _stream(2, seed=3)
    srv = serve.Server(n_slots=2, hbm_budget=1 << 20)
    with pytest.raises(ValueError, match="budget"):
        srv.run(jobs)
