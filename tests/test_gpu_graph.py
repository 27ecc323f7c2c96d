"""Long step calls of a single case replay captured runs of steps (a
hipGraph per buffer set) and launch the rest one by one: the state equals
that of the same steps launched one call at a time, bit for bit, in Mode H
and in the divided cavity, also after a setting the captured launches hold
(the physics, a wall, the rows per wave) changes between calls."""
import numpy as np
import pytest

from synth_inputs import perturbation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def _same(a, b):
    for f in ("u", "v", "T"):
        x, y = a.fetch(f), b.fetch(f)
        assert np.array_equal(x, y), (f, np.abs(x - y).max())


@pytest.mark.parametrize("mode,prec,nx,ny", [(0, "f32", 130, 70), (0, "f64", 64, 64),
                                             (1, "f32", 96, 40), (1, "f64", 64, 32)])
def test_graph_runs_equal_single_launches(lf, ctx, mode, prec, nx, ny):
    T0 = perturbation(nx, ny, 91, amp=0.05)
    mk = lambda: lf.Case(ctx, nx, ny, prec, mode=mode).set_physics(2e5, 0.71).set_cavity_walls().init(T0)
    a, b = mk(), mk()
    a.step(301)  # four captured runs of 64 steps, then 45 single steps
    for _ in range(301):
        b.step(1)
    assert a.steps == b.steps == 301
    _same(a, b)
    # settings held by the captured launches change: captured again
    for c in (a, b):
        c.set_physics(5e4, 7.0)
    a.step(200)
    for _ in range(200):
        b.step(1)
    _same(a, b)
    for c in (a, b):
        c.set_wall(lf.S, lf.WALL_NOSLIP, 0.0, lf.T_DIRICHLET, 0.25)
    a.step(130)
    for _ in range(130):
        b.step(1)
    _same(a, b)
    if mode == 0:
        ctx.set_band(2)
        try:
            a.step(129)
            for _ in range(129):
                b.step(1)
        finally:
            ctx.set_band(0)
        _same(a, b)
    assert a.nusselt() == b.nusselt()
