"""GPU parity of Mode H on grid setting 2 (coarse temperature control volumes
under the lattice, one implicit energy step per S lattice steps, Sec. 5.1)
against the FP64 numpy oracle, through the C-ABI library."""
import os

import numpy as np
import pytest

from oracle.gs2 import GS2Case
from synth_inputs import perturbation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def restrict(T0):
    """Each control volume starts at the mean of its 2 x 2 nodes."""
    return 0.25 * ((T0[0::2, 0::2] + T0[0::2, 1::2]) + (T0[1::2, 0::2] + T0[1::2, 1::2]))


def pair(lf, ctx, nx, ny, prec, S=0, K=0, Ra=1e5, Pr=0.71, T0=None):
    g = lf.Case(ctx, nx, ny, prec, mode=lf.MODE_HYBRID_GS2).set_physics(Ra, Pr).set_cavity_walls()
    if S or K:
        g.set_subcycle(S, K)
    g.init(T0)
    o = GS2Case(nx, ny, S=S, K=K or 4).set_physics(Ra, Pr)
    o.init(None if T0 is None else restrict(T0))
    assert abs(g.params()["nu"] - o.params["nu"]) < 1e-15
    return g, o


def rel_linf(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def check(g, o, tol, fields=("u", "v", "T", "rho")):
    errs = {}
    for f in fields:
        a, b = g.fetch(f), o.fetch(f)
        errs[f] = rel_linf(a - (1 if f == "rho" else 0), b - (1 if f == "rho" else 0))
    for f, e in errs.items():
        assert e <= tol, (f, e, errs)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= tol * abs(no[k]), (k, ng[k], no[k])
    return errs


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_gs2_parity_default_cycle(lf, ctx, prec, tol):
    """40 x 24 lattice, 20 x 12 control volumes, S = 2NX = 40, K = 4:
    ten energy steps."""
    nx, ny = 40, 24
    T0 = perturbation(nx, ny, 51, amp=0.1)
    g, o = pair(lf, ctx, nx, ny, prec, T0=T0)
    g.step(400)
    o.step(400)
    check(g, o, tol)


def test_gs2_parity_ragged_short_cycle(lf, ctx):
    """136 x 72 (several blocks and line batches per direction), S = 17,
    K = 3, Ra 1e6, twenty energy steps, FP64."""
    nx, ny = 136, 72
    T0 = perturbation(nx, ny, 52, amp=0.1)
    g, o = pair(lf, ctx, nx, ny, "f64", S=17, K=3, Ra=1e6, T0=T0)
    g.step(340)
    o.step(340)
    check(g, o, 1e-10)


def test_gs2_cycle_phase_survives_split_calls(lf, ctx):
    """The energy step follows every S-th lattice step counted since init,
    however the steps are split across calls."""
    nx, ny = 32, 16
    T0 = perturbation(nx, ny, 53, amp=0.1)
    a = lf.Case(ctx, nx, ny, "f64", mode=lf.MODE_HYBRID_GS2).set_physics(1e5, 0.71)
    a.set_cavity_walls().set_subcycle(10, 2).init(T0)
    b = lf.Case(ctx, nx, ny, "f64", mode=lf.MODE_HYBRID_GS2).set_physics(1e5, 0.71)
    b.set_cavity_walls().set_subcycle(10, 2).init(T0)
    a.step(47)
    for n in (3, 9, 1, 20, 14):
        b.step(n)
    for f in ("u", "v", "T"):
        assert np.array_equal(a.fetch(f), b.fetch(f)), f


def test_gs2_conduction_limit(lf, ctx):
    """g beta = 0: the linear profile and Nu = 1/A to rounding."""
    nx, ny = 32, 16
    g = lf.Case(ctx, nx, ny, "f64", mode=lf.MODE_HYBRID_GS2).set_lattice(0.05, 0.1, 0.0)
    g.set_cavity_walls().init()
    g.step(32 * 300)
    lin = 0.5 - (np.arange(nx) + 0.5) / nx
    assert np.abs(g.fetch("T") - lin[None, :]).max() < 1e-12
    assert abs(g.nusselt()["nu_hot"] - ny / nx) < 1e-11


def test_gs2_errors(lf, ctx):
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 34, 17, mode=lf.MODE_HYBRID_GS2)
    assert e.value.status == lf.LF_EINVAL
    h = lf.Case(ctx, 32, 16)
    with pytest.raises(lf.LFError) as e:
        h.set_subcycle(8, 2)
    assert e.value.status == lf.LF_EINVAL
    g = lf.Case(ctx, 32, 16, mode=lf.MODE_HYBRID_GS2)
    with pytest.raises(lf.LFError) as e:
        g.set_subcycle(-1, 2)
    assert e.value.status == lf.LF_EINVAL


GOLDEN_GS2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gs2_steady_64.npz")


@pytest.mark.parametrize("prec,tol", [("f64", 1e-8), ("f32", 1e-4)])
def test_gs2_steady_state_against_the_exact_implicit_step(lf, ctx, prec, tol):
    """The library relaxes each implicit energy step by 4 line sweeps; a
    fixed point of the sweeps solves the whole step, so its steady state is
    the exact step's.  64 x 64 lattice (32 x 32 control volumes), Ra 1e4,
    from rest, run to steady (checks every 16 energy cycles; FP64 to a
    1e-12 change, FP32 to its own stop rule) against the oracle's steady
    state with every energy step solved exactly (sparse direct solve,
    tests/golden/gs2_steady_64.npz)."""
    if not os.path.exists(GOLDEN_GS2):
        pytest.skip("golden steady state not generated")
    gd = np.load(GOLDEN_GS2)
    c = lf.Case(ctx, 64, 64, prec, mode=lf.MODE_HYBRID_GS2).set_physics(1e4, 0.71)
    c.set_cavity_walls().init()
    steps, r, rule = c.run_to_steady(tol=1e-12 if prec == "f64" else 1e-8, check_every=1024,
                                     max_steps=2_000_000)
    for f in ("u", "v", "T"):
        assert rel_linf(c.fetch(f), gd[f]) <= tol, (prec, f, steps, r, rule)
    nu = c.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(nu[k] - float(gd[k])) <= tol * abs(float(gd[k])), (prec, k, nu[k])
