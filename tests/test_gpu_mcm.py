"""GPU LBM-MCM (Sec. 6) against the oracle: the walkers of sampled nodes
replayed one by one on the CPU (same splitmix64 streams, decisions in FP64)
must give the library's node temperatures exactly; the whole field must
lie within the estimator's standard error of its expectation (the linear
system of Eq 97); the coupled run must track the deterministic reference."""
import numpy as np
import pytest

from oracle.mcm import MCMCase, exact_expectation, walk
from synth_inputs import perturbation

pytestmark = pytest.mark.gpu

SEED = 1908083869


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def case(lf, ctx, nx, ny, prec, S, N, Ra=1e4, T0=None, max_steps=1 << 20):
    g = lf.Case(ctx, nx, ny, prec, mode=lf.MODE_LBM_MCM).set_physics(Ra, 0.71).set_cavity_walls()
    g.set_mcm(S, N, SEED, max_steps).init(T0)
    return g


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_solve_replays_exactly_and_estimates_the_expectation(lf, ctx, prec):
    nx, ny, S, N = 24, 20, 60, 256
    T0 = perturbation(nx, ny, 71, amp=0.3)
    g = case(lf, ctx, nx, ny, prec, S, N, T0=T0)
    g.step(S)  # lattice steps, then the first Monte Carlo solve (stream seed SEED + 0)
    assert g.mcm_capped() == 0
    u, v, T = g.fetch("u"), g.fetch("v"), g.fetch("T")
    al = g.params()["alpha"]
    if prec == "f32":
        al = float(np.float32(al))  # the kernel reads alpha in the working precision
    tfix, Tw = [1, 1, 0, 0], [0.5, -0.5, 0.0, 0.0]
    for (i, j) in ((0, 0), (11, 9), (23, 19), (5, 14)):
        rec = [walk(i, j, w, N, SEED, u, v, al, tfix, Tw, 1 << 20)[0] for w in range(N)]
        est = np.mean(rec)
        if prec == "f32":
            est = float(np.float32(est))
        assert T[j, i] == est, (i, j, T[j, i], est)
    ref = exact_expectation(u, v, al, tfix, Tw)
    err = np.abs(T - ref)
    se = 0.5 / np.sqrt(N)
    assert err.max() <= 5.5 * se and err.mean() <= 1.0 * se, (err.max() / se, err.mean() / se)


def test_coupled_run_tracks_the_reference(lf, ctx):
    """32 x 32, Ra 1e4, one solve of 16384 walkers per node every 100
    lattice steps, 3000 steps: the wall-averaged Nusselt numbers within 3 %
    (about three standard errors of the estimator) and the maximum within
    8 % of the deterministic reference (the walkers' expectation)."""
    n, S, N = 32, 100, 16384
    g = case(lf, ctx, n, n, "f32", S, N)
    o = MCMCase(n, n, S=S).set_physics(1e4, 0.71).init()
    g.step(3000)
    o.step(3000)
    assert g.mcm_capped() == 0
    ng, no = g.nusselt(), o.nusselt()
    for k, tol in (("nu_hot", 0.03), ("nu_cold", 0.03), ("nu_hot_max", 0.08)):
        assert abs(ng[k] - no[k]) <= tol * abs(no[k]), (k, ng[k], no[k])


def test_mcm_errors(lf, ctx):
    h = lf.Case(ctx, 16, 16)
    with pytest.raises(lf.LFError) as e:
        h.set_mcm(10, 8)
    assert e.value.status == lf.LF_EINVAL
    g = lf.Case(ctx, 16, 16, mode=lf.MODE_LBM_MCM)
    with pytest.raises(lf.LFError) as e:
        g.set_mcm(0, 8)
    assert e.value.status == lf.LF_EINVAL
    # all walls adiabatic: no wall can absorb a walker
    g.set_physics(1e4, 0.71)
    for side in (lf.W, lf.E, lf.S, lf.N):
        g.set_wall(side, lf.WALL_NOSLIP, 0.0, lf.T_ADIABATIC, 0.0)
    g.set_mcm(2, 8).init()
    with pytest.raises(lf.LFError) as e:
        g.step(2)
    assert e.value.status == lf.LF_EINVAL
