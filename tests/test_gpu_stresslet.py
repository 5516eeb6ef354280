"""Combined single and double layer sources (Stokeslet + stresslet, Sec. 2.3) on the GPU.

Stage parity against the spectral oracle (element by element, 1e-12 / 1e-11 relative to the
array's max, plans with tol < 1e-10 so the full-precision pair formula runs), the whole sum
against the classical Ewald oracle within tol, and the structure of the entry point."""
import numpy as np
import pytest

import oracle
from oracle import spectral as S
from paper_2606_19059_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (box, grid, xi, r_c, P, m)
CASES = {
    "cube32_P8": ((1.0, 1.0, 1.0), (32, 32, 32), 11.44, 0.387, 8, 4.8),
    "aniso_P12": ((1.0, 1.3, 0.8), (16, 32, 64), 9.0, 0.30, 12, 5.8),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def sources(n, box, seed):
    x, f = W.particles(n, box, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    return x, f, rng.standard_normal((3, n)), rng.standard_normal((3, n))


@pytest.mark.parametrize("name,n", [("cube32_P8", 1500), ("aniso_P12", 1201)])
def test_combined_stages_match_spectral_oracle(name, n):
    import paper_2606_19059_amd as E

    box, grid, xi, rc, P, m = CASES[name]
    pl = E.Plan(box, 1e-11, xi=xi, r_c=rc, grid=grid, P=P, window_shape=m, n_max=n, stresslet=True)
    x, f, q, nr = sources(n, box, seed=41)
    un, uf = pl.eval_combined_parts(dev(x), dev(f), dev(q), dev(nr))
    St = oracle.stresslet_tensor(q, nr)
    ref_n = oracle.real_space(x, f, box, xi, rc) + oracle.real_space_st(x, St, box, xi, rc)
    ref_f = S.far_field_combined(x, f, St, box, grid, xi, P, m)
    assert maxrel(host(un), ref_n) < 1e-12
    assert maxrel(host(uf), ref_f) < 1e-11
    u = host(pl.eval_combined(dev(x), dev(f), dev(q), dev(nr)))
    assert maxrel(u, S.spectral_ewald(x, f, box, grid, xi, rc, P, m, q=q, nrm=nr)) < 1e-11


def test_stresslet_only_and_linearity():
    """Combined = Stokeslet alone + stresslet alone; zero stresslets reproduce ewald_eval."""
    import paper_2606_19059_amd as E

    box, grid, xi, rc, P, m = CASES["cube32_P8"]
    pl = E.Plan(box, 1e-11, xi=xi, r_c=rc, grid=grid, P=P, window_shape=m, n_max=900, stresslet=True)
    x, f, q, nr = sources(900, box, seed=42)
    X, F, Q, N = dev(x), dev(f), dev(q), dev(nr)
    z = torch.zeros_like(X)
    both = host(pl.eval_combined(X, F, Q, N))
    only_f = host(pl.eval_combined(X, F, z, z))
    only_s = host(pl.eval_combined(X, z, Q, N))
    assert maxrel(only_f, host(pl.eval(X, F))) < 1e-13
    assert maxrel(only_f + only_s, both) < 1e-12
    # the stresslet part alone against the classical oracle at the plan's accuracy
    ref = oracle.ewald_sum(x, np.zeros_like(f), box, q=q, nrm=nr)
    assert oracle.rel_err(only_s, ref) < 1e-5


@pytest.mark.parametrize("tol,precision", [(1e-4, "fp32"), (1e-6, "fp32"), (1e-6, "fp64"), (1e-8, "fp64")])
def test_combined_sum_meets_tolerance(tol, precision):
    """Plans derived from tol alone (cost model, Stokeslet error split) against the classical
    Ewald oracle of the combined sum."""
    import paper_2606_19059_amd as E

    box = (1.0, 1.0, 1.0)
    x, f, q, nr = sources(2000, box, seed=43)
    pl = E.Plan(box, tol, n_max=2000, precision=precision, stresslet=True)
    u = host(pl.eval_combined(dev(x), dev(f), dev(q), dev(nr)))
    err = oracle.rel_err(u, oracle.ewald_sum(x, f, box, q=q, nrm=nr))
    print("combined %s tol %g grid %s P %d: err %.3e" % (precision, tol, pl.info["grid"], pl.info["P"], err))
    assert err <= tol


def test_combined_entry_point_errors():
    import paper_2606_19059_amd as E

    box, grid, xi, rc, P, m = CASES["cube32_P8"]
    x, f, q, nr = sources(50, box, seed=44)
    plain = E.Plan(box, 1e-6, xi=xi, r_c=rc, grid=grid, P=P, window_shape=m, n_max=50)
    with pytest.raises(E.EwaldError) as ei:
        plain.eval_combined(dev(x), dev(f), dev(q), dev(nr))
    assert ei.value.code == E.EWALD_EINVAL


def test_combined_empty_and_single_particle():
    """n = 0 is a no-op; one particle's stresslet sees only its own periodic images."""
    import paper_2606_19059_amd as E

    box = (1.0, 1.0, 1.0)
    pl = E.Plan(box, 1e-8, grid=(32, 32, 32), n_max=4, stresslet=True)
    z = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    assert pl.eval_combined(z, z, z, z).shape == (3, 0)
    x = np.array([[0.3], [0.6], [0.1]])
    f = np.array([[0.2], [-0.4], [1.0]])
    q = np.array([[1.0], [0.5], [-0.3]])
    nr = np.array([[0.2], [-1.0], [0.4]])
    u = host(pl.eval_combined(dev(x), dev(f), dev(q), dev(nr)))
    assert oracle.rel_err(u, oracle.ewald_sum(x, f, box, q=q, nrm=nr)) < 1e-7
