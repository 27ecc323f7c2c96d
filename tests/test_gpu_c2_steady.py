"""The 512 x 512 side-heated cavity at Ra 1e6, Pr 0.71 against the FP64
oracle's steady state, stored by tests/golden/make_c2_steady.py.

The GPU runs exactly the oracle's step count S_o from the same seeded T0 and
is compared with it: the FP64 path on every 4th node (the stored FP64
samples) and on the wall columns to 1e-9 of the field maxima; the FP32 path
(shifted populations, compensated T) on every node (the stored field rounded
to FP32, which moves it by less than 1e-7 of the maxima) to 1e-4; the
Nusselt numbers to 1e-9 / 1e-4.  At this size the slowest modes decay by
only ~1e-5 per step, which amplifies FP32 rounding that is coherent over
regions of nodes into the fixed point; the collision's equilibrium is formed
so that it carries none (measured at S_o over every node: u 3.7e-6, v 2.0e-6, T 8.4e-7 of
the maxima).  Then the FP32 path runs to its own stop (residual 1e-8 or the
FP32 floor rule) and its Nusselt number is compared with the oracle's."""
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


TOL = {"f64": (1e-9, 1e-9), "f32": (1e-4, 1e-4)}  # (fields, Nusselt numbers)


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
    for name, a, m in (("u", u, mx[0]), ("v", v, mx[1]), ("T", T, mx[2])):
        if prec == "f64":
            e = np.abs(a[::4, ::4] - golden[name + "_s"]).max() / m
        else:
            e = np.abs(a - golden[name + "32"].astype(np.float64)).max() / m
        print(f"{prec} {name}: max error {e:.2e} of the field maximum", flush=True)
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
