"""Batched Mode H cavities: parity with the oracle per cavity, bitwise
equality with the same cavity run alone, graph replays equal to eager
stepping, per-cavity run to steady state, autotuner."""
import json
import os

import numpy as np
import pytest

import oracle
from synth_inputs import cavity_sweep, perturbation

pytestmark = pytest.mark.gpu

CASES = [
    dict(nx=64, ny=64, Ra=1e4, Pr=0.71, seed=1),
    dict(nx=96, ny=48, Ra=1e5, Pr=7.0, seed=2),
    dict(nx=130, ny=40, Ra=3e4, Pr=0.71, seed=3),
    dict(nx=70, ny=66, Ra=2e5, Pr=0.71, seed=4),
    dict(nx=128, ny=32, Ra=1e3, Pr=7.0, seed=5),
]


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def T0_of(c, amp=0.05):
    return perturbation(c["nx"], c["ny"], c["seed"], amp=amp)


def rel_linf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_batch_matches_oracle_per_cavity(lf, ctx, prec, tol):
    oracle.set_threads(8)
    b = lf.Batch(ctx, CASES, prec).init([T0_of(c) for c in CASES])
    b.step(400)
    for k, c in enumerate(CASES):
        o = oracle.Case(c["nx"], c["ny"]).set_physics(c["Ra"], c["Pr"]).set_cavity_walls()
        o.init(T0_of(c)).step(400)
        assert abs(b.params(k)["nu"] - o.params["nu"]) < 1e-15
        for f in ("u", "v", "T"):
            e = rel_linf(b.fetch(k, f), o.fetch(f))
            assert e <= tol, (k, f, e)
        assert abs(b.nusselt(k)["nu_hot"] - o.nusselt()["nu_hot"]) <= tol * o.nusselt()["nu_hot"]


def test_batch_member_equals_solo_bitwise(lf, ctx):
    b = lf.Batch(ctx, CASES, "f32").init([T0_of(c) for c in CASES])
    b.set_band(3)
    b.step(250)
    for k, c in enumerate(CASES):
        s = lf.Case(ctx, c["nx"], c["ny"], "f32").set_physics(c["Ra"], c["Pr"])
        s.set_cavity_walls().init(T0_of(c)).step(250)
        for f in ("u", "v", "T"):
            assert np.array_equal(b.fetch(k, f), s.fetch(f)), (k, f)


def test_graph_replays_equal_eager_steps(lf, ctx):
    K = 100
    g = lf.Batch(ctx, CASES, "f32").init([T0_of(c) for c in CASES])
    e = lf.Batch(ctx, CASES, "f32").init([T0_of(c) for c in CASES])
    for rep in range(3):
        # one replay of the captured "K steps + residual" graph per call
        g.run_to_steady(tol=1e-30, check_every=K, max_steps=(rep + 1) * K,
                        raise_on_notconv=False)
        g.reactivate()
        e.step(K)
        re = e.residual()
        ctx.stream.synchronize()
        for k in range(len(CASES)):
            for f in ("u", "v", "T"):
                assert np.array_equal(g.fetch(k, f), e.fetch(k, f)), (rep, k, f)
        assert np.all(np.isfinite(re))


def test_batch_run_to_steady_fp64_matches_oracle(lf, ctx):
    oracle.set_threads(8)
    cases = [dict(nx=32, ny=32, Ra=1e4, Pr=0.71, seed=0),
             dict(nx=48, ny=24, Ra=1e3, Pr=7.0, seed=0),
             dict(nx=40, ny=40, Ra=5e4, Pr=0.71, seed=0)]
    b = lf.Batch(ctx, cases, "f64").init()
    steps, rules, r = b.run_to_steady(tol=1e-8, check_every=1000, max_steps=400000)
    assert np.all(rules == lf.STOP_TOL), rules
    for k, c in enumerate(cases):
        o = oracle.Case(c["nx"], c["ny"]).set_physics(c["Ra"], c["Pr"]).set_cavity_walls().init()
        so, ro = o.run_to_steady(tol=1e-8, check_every=1000, max_steps=400000)
        assert steps[k] == so, (k, steps[k], so)
        nb, no = b.nusselt(k), o.nusselt()
        for key in ("nu_hot", "nu_cold", "nu_hot_max"):
            assert abs(nb[key] - no[key]) <= 1e-9 * abs(no[key]), (k, key)


def test_batch_run_to_steady_fp32_sweep_sample(lf, ctx):
    """Eight cavities of the sweep distribution, capped at 64 rows, FP32:
    each stops by the tolerance or the FP32 floor rule, with Nu within 1e-4
    of the FP64 oracle's steady value."""
    oracle.set_threads(8)
    cases = cavity_sweep(8, max_ny=64)
    b = lf.Batch(ctx, cases, "f32").init()
    steps, rules, r = b.run_to_steady(tol=1e-8, check_every=1000, max_steps=600000)
    assert np.all((rules == lf.STOP_TOL) | (rules == lf.STOP_FLOOR)), (rules, r)
    for k, c in enumerate(cases):
        o = oracle.Case(c["nx"], c["ny"]).set_physics(c["Ra"], c["Pr"]).set_cavity_walls().init()
        o.run_to_steady(tol=1e-8, check_every=1000, max_steps=600000)
        nb, no = b.nusselt(k)["nu_hot"], o.nusselt()["nu_hot"]
        assert abs(nb - no) <= 1e-4 * abs(no), (k, c, nb, no, steps[k], rules[k], r[k])


def test_run_to_steady_resumes_after_step_limit(lf, ctx):
    """A run split into calls with growing max_steps equals one call."""
    cases = [dict(nx=32, ny=32, Ra=1e4, Pr=0.71, seed=0), dict(nx=48, ny=24, Ra=1e3, Pr=7.0, seed=0)]
    one = lf.Batch(ctx, cases, "f64").init()
    s1, r1, _ = one.run_to_steady(tol=1e-8, check_every=1000, max_steps=400000)
    two = lf.Batch(ctx, cases, "f64").init()
    sa, ra, _ = two.run_to_steady(tol=1e-8, check_every=1000, max_steps=6000,
                                  raise_on_notconv=False)
    assert np.all(ra == 0) and np.all(sa == 6000)
    s2, r2, _ = two.run_to_steady(tol=1e-8, check_every=1000, max_steps=400000)
    assert np.array_equal(s1, s2) and np.array_equal(r1, r2)
    for k in range(2):
        for f in ("u", "v", "T"):
            assert np.array_equal(one.fetch(k, f), two.fetch(k, f)), (k, f)


def test_autotuner_writes_and_loads_cache(lf, ctx, tmp_path):
    path = str(tmp_path / "tune.json")
    table = ctx.autotune(path, budget_ms=1400, scratch_bytes=1 << 30)
    assert sorted(table) == [64, 96, 128, 192, 256, 384, 512]
    assert set(table.values()) <= {1, 2, 4, 8, 16}
    d = json.load(open(path))
    assert d["arch"] == "gfx950" and d["precision"] == "f32"
    ctx2 = lf.Context(0)
    assert ctx2.autotune(path) == table  # loaded, not re-measured


def test_batch_errors(lf, ctx):
    b = lf.Batch(ctx, CASES[:2], "f32").init()
    with pytest.raises(lf.LFError) as e:
        b.run_to_steady(check_every=999)
    assert e.value.status == lf.LF_EINVAL
    # a cavity whose nine FP64 planes exceed the step kernel's 32-bit byte range
    big = {"nx": 8192, "ny": 8192, "Ra": 1e6, "Pr": 0.71}
    with pytest.raises(lf.LFError) as e:
        lf.Batch(ctx, [CASES[0], big], "f64")
    assert e.value.status == lf.LF_EINVAL


def first_of_each_class(sweep):
    """Draw index of the first cavity of every (ny, aspect) class."""
    seen = {}
    for k, c in enumerate(sweep):
        seen.setdefault((c["ny"], c["aspect"]), k)
    return sorted(seen.values())


def test_sweep_classes_against_the_oracle(lf, ctx):
    """The first cavity of each of the 28 (ny, aspect) classes of the
    256-cavity sweep (ny 64 .. 512, aspect 1 .. 4, the largest 2048 x 512
    among them; 5.4 M nodes), stepped together as one FP32 batch for 1000
    steps from their seeded T0, each against the FP64 oracle element by
    element: u, v, T and the Nusselt numbers within 1e-4."""
    sweep = cavity_sweep(256)
    picks = first_of_each_class(sweep)
    assert len(picks) == 28 and 35 in picks  # draw 35 is the 2048 x 512 cavity
    cases = [sweep[k] for k in picks]
    T0 = [perturbation(c["nx"], c["ny"], c["seed"]) for c in cases]
    b = lf.Batch(ctx, cases, "f32").init(T0)
    b.step(1000)
    oracle.set_threads(16)
    for k, c in enumerate(cases):
        print(f"sweep class ny {c['ny']} aspect {c['aspect']} (draw {picks[k]})", flush=True)
        o = oracle.Case(c["nx"], c["ny"]).set_physics(c["Ra"], c["Pr"]).set_cavity_walls()
        o.init(T0[k]).step(1000)
        assert abs(b.params(k)["nu"] - o.params["nu"]) < 1e-15
        for f in ("u", "v", "T"):
            e = rel_linf(b.fetch(k, f), o.fetch(f))
            assert e <= 1e-4, (picks[k], f, e)
        nb, no = b.nusselt(k), o.nusselt()
        for key in ("nu_hot", "nu_cold"):
            assert abs(nb[key] - no[key]) <= 1e-4 * abs(no[key]), (picks[k], key)
    b.close()


GOLDEN_SWEEP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                            "sweep_steady_64.npz")


def test_smallest_sweep_cavities_to_steady_state(lf, ctx):
    """The three ny = 64 classes of the sweep (aspect 1, 2, 3), run together
    as one FP32 batch to steady state by the library's own stop rule (1e-8,
    or the FP32 floor once the slowest mode has settled), against the FP64
    oracle's steady state (residual 1e-8; tests/golden/sweep_steady_64.npz):
    u, v, T and the Nusselt numbers within 1e-4."""
    if not os.path.exists(GOLDEN_SWEEP):
        pytest.skip("golden steady states not generated")
    gd = np.load(GOLDEN_SWEEP)
    sweep = cavity_sweep(256)
    draws = [int(k) for k in gd["draws"]]
    cases = [sweep[k] for k in draws]
    b = lf.Batch(ctx, cases, "f32").init([perturbation(c["nx"], c["ny"], c["seed"])
                                          for c in cases])
    steps, rules, r = b.run_to_steady(tol=1e-8, check_every=1000, max_steps=5_000_000)
    for i, k in enumerate(draws):
        print(f"draw {k}: {steps[i]} steps (oracle {int(gd[f'steps_{k}'])}), rule {rules[i]}",
              flush=True)
        assert rules[i] in (lf.STOP_TOL, lf.STOP_FLOOR)
        for f in ("u", "v", "T"):
            e = rel_linf(b.fetch(i, f), gd[f"{f}_{k}"].astype(np.float64))
            assert e <= 1e-4, (k, f, e)
        nu = b.nusselt(i)
        ref = gd[f"nu_{k}"]
        assert abs(nu["nu_hot"] - ref[0]) <= 1e-4 * abs(ref[0]), k
        assert abs(nu["nu_cold"] - ref[1]) <= 1e-4 * abs(ref[1]), k
    b.close()
