"""The 512 x 512 side-heated cavity at Ra 1e6, Pr 0.71 against the FP64
oracle's steady state, stored by tests/golden/make_c2_steady.py.

The GPU runs exactly the oracle's step count S_o from the same seeded T0 and
is compared on every 4th node, on both wall columns and on the Nusselt
numbers: the FP64 path to 1e-9; the FP32 path (shifted populations,
compensated T) to 1e-4 on the Nusselt numbers and 5e-4 on the fields.  At
this size the slowest modes decay by ~1e-5 per step, which amplifies FP32
rounding noise in the fixed point (measured at S_o: u 4.3e-4, v 1.9e-4,
T 1.4e-4, Nu 4.9e-5 of the field maxima; FP64: 5e-11).  Then the FP32 path
runs to its own stop (residual 1e-8 or the FP32 floor rule) and its
Nusselt number is compared with the oracle's."""
import os

import numpy as np
import pytest

from synth_inputs import SEED_C2, perturbation

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_steady_512.npz")
KEYS = ("nu_hot", "nu_cold", "nu_hot_max", "y_hot_max", "nu_cold_max", "y_cold_max",
        "nu_hot_o2", "nu_cold_o2")


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden steady state not generated")
    return np.load(GOLDEN)


TOL = {"f64": (1e-9, 1e-9), "f32": (5e-4, 1e-4)}  # (fields, Nusselt numbers)


@pytest.fixture(scope="module", params=["f64", "f32"])
def case(request, golden):
    import paper_1908_08386_amd as lf
    ctx = lf.Context(0)
    n = 512
    c = lf.Case(ctx, n, n, request.param).set_physics(1e6, 0.71).set_cavity_walls()
    c.init(perturbation(n, n, SEED_C2))
    c.step(int(golden["steps"]))
    return request.param, c


def test_fields_at_oracle_step_count(golden, case):
    prec, c = case
    tol = TOL[prec][0]
    u, v, T = c.fetch("u"), c.fetch("v"), c.fetch("T")
    mx = golden["max_abs"]
    for name, a, ref, m in (("u", u, golden["u_s"], mx[0]), ("v", v, golden["v_s"], mx[1]),
                            ("T", T, golden["T_s"], mx[2])):
        e = np.abs(a[::4, ::4] - ref).max() / m
        assert e <= tol, (prec, name, e)
    for name, a, ref in (("T_west", T[:, 0], golden["T_west"]), ("T_east", T[:, -1], golden["T_east"])):
        assert np.abs(a - ref).max() <= tol * mx[2], (prec, name)


def test_nusselt_at_oracle_step_count(golden, case):
    prec, c = case
    tol = TOL[prec][1]
    nu = c.nusselt()
    ref = dict(zip(KEYS, golden["nusselt"]))
    for k in ("nu_hot", "nu_cold", "nu_hot_max", "nu_cold_max", "nu_hot_o2", "nu_cold_o2"):
        assert abs(nu[k] - ref[k]) <= tol * abs(ref[k]), (prec, k, nu[k], ref[k])
    for k in ("y_hot_max", "y_cold_max"):
        assert abs(nu[k] - ref[k]) <= 1.0 / 512 + 1e-12, (prec, k)


def test_own_stop_rule_reaches_the_oracle_nusselt(golden):
    import paper_1908_08386_amd as lf
    ctx = lf.Context(0)
    n = 512
    c = lf.Case(ctx, n, n, "f32").set_physics(1e6, 0.71).set_cavity_walls()
    c.init(perturbation(n, n, SEED_C2))
    steps, r, rule = c.run_to_steady(tol=1e-8, check_every=1000, max_steps=6_000_000)
    assert rule in (lf.STOP_TOL, lf.STOP_FLOOR)
    ref = dict(zip(KEYS, golden["nusselt"]))
    assert abs(c.nusselt()["nu_hot"] - ref["nu_hot"]) <= 1e-4 * ref["nu_hot"], (steps, r, rule)
