"""GPU parity of the domain-decomposed mode (LBM west half, FV east half)
against the FP64 oracle, through the C-ABI library."""
import numpy as np
import pytest

import oracle
from synth_inputs import perturbation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import paper_1908_08386_amd as lf
    return lf


@pytest.fixture(scope="module")
def ctx(lf):
    return lf.Context(0)


def rel_linf(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def pair(lf, ctx, nx, ny, prec, iface, Ra=1e5, Pr=0.71, T0=None):
    g = lf.Case(ctx, nx, ny, prec, mode=lf.MODE_SPLIT, iface=iface)
    g.set_physics(Ra, Pr).set_cavity_walls().init(T0)
    o = oracle.DDCase(nx, ny, oracle.SPLIT, iface).set_physics(Ra, Pr).set_cavity_walls()
    o.init(T0)
    assert abs(g.params()["nu"] - o.params["nu"]) < 1e-15
    return g, o


def check(g, o, tol, fields=("u", "v", "T", "rho")):
    errs = {}
    for f in fields:
        a, b = g.fetch(f), o.fetch(f)
        errs[f] = rel_linf(a - (1 if f == "rho" else 0), b - (1 if f == "rho" else 0))
    for f, e in errs.items():
        assert e <= tol, (f, e, errs)
    return errs


@pytest.mark.parametrize("iface", [0, 1])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_split_parity_small(lf, ctx, iface, prec, tol):
    oracle.set_threads(8)
    nx, ny = 64, 48
    T0 = perturbation(nx, ny, 31, amp=0.1)
    g, o = pair(lf, ctx, nx, ny, prec, iface, T0=T0)
    g.step(600)
    o.step(600)
    check(g, o, tol)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= tol * abs(no[k]), k


def test_split_parity_ragged_fp64(lf, ctx):
    oracle.set_threads(8)
    nx, ny = 138, 77  # split column 69: the LBM and FV zones span ragged tiles
    T0 = perturbation(nx, ny, 32, amp=0.05)
    g, o = pair(lf, ctx, nx, ny, "f64", 0, Ra=1e6, T0=T0)
    for _ in range(3):
        g.step(300)
        o.step(300)
        np.testing.assert_allclose(g.residual(), o.residual(), rtol=1e-8)
    check(g, o, 1e-10)


@pytest.mark.parametrize("conv,prec,tol", [(0, "f64", 1e-10), (1, "f64", 1e-10), (2, "f64", 1e-10),
                                           (0, "f32", 1e-4)])
def test_split_parity_inner_waves(lf, ctx, conv, prec, tol):
    """A FV zone wide enough for the interior (direct-addressed) path: 201 FV
    columns, of which the waves starting at columns 263 and 327 take it, with
    ragged rows; each convection scheme against the oracle."""
    oracle.set_threads(8)
    nx, ny = 400, 70
    T0 = perturbation(nx, ny, 33, amp=0.1)
    g = lf.Case(ctx, nx, ny, prec, mode=lf.MODE_SPLIT, iface=0)
    g.set_physics(1e5, 0.71, conv=conv).set_cavity_walls().init(T0)
    o = oracle.DDCase(nx, ny, oracle.SPLIT, 0).set_physics(1e5, 0.71).set_cavity_walls()
    o.set_lattice(o.params["nu"], o.params["alpha"], o.params["gbeta"], 0.0, conv=conv)
    o.init(T0)
    g.step(400)
    o.step(400)
    check(g, o, tol)


def test_split_128_fp32_2000_steps(lf, ctx):
    oracle.set_threads(8)
    n = 128
    g, o = pair(lf, ctx, n, n, "f32", 0, Ra=1e6, T0=perturbation(n, n, 1908083860))
    g.step(2000)
    o.step(2000)
    check(g, o, 1e-4, ("u", "v", "T"))


def test_split_conduction_limit(lf, ctx):
    nx, ny = 40, 16
    g = lf.Case(ctx, nx, ny, "f64", mode=lf.MODE_SPLIT).set_lattice(0.05, 0.15, 0.0)
    g.set_cavity_walls().init()
    g.step(30000)
    lin = np.tile(0.5 - (np.arange(nx) + 0.5) / nx, (ny, 1))
    assert np.abs(g.fetch("T") - lin).max() < 1e-9
    assert np.abs(g.fetch("u")).max() < 1e-12
    assert abs(g.nusselt()["nu_hot"] - ny / nx) < 1e-8


def test_split_errors(lf, ctx):
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 65, 32, mode=lf.MODE_SPLIT)
    assert e.value.status == lf.LF_EINVAL
    g = lf.Case(ctx, 64, 32, mode=lf.MODE_SPLIT)
    with pytest.raises(lf.LFError) as e:
        g.set_lattice(0.09, 0.05)  # above the FV zone's nu <= 1/12 bound
    assert e.value.status == lf.LF_EUNSTABLE
    with pytest.raises(lf.LFError) as e:
        g.set_wall(lf.S, lf.WALL_PERIODIC, 0.0, lf.T_PERIODIC, 0.0)
    assert e.value.status == lf.LF_ENOTIMPL


def test_split_full_size_first_steps(lf, ctx):
    """4096 x 4096 split cavity, Ra 1e6, FP32, in the benchmark's launch
    configuration: element-wise parity with the oracle over the first steps."""
    oracle.set_threads(16)
    n = 4096
    g, o = pair(lf, ctx, n, n, "f32", 0, Ra=1e6, T0=perturbation(n, n, 1908083860))
    g.step(4)
    o.step(4)
    check(g, o, 1e-4, ("T",))
    # velocities start from rest: compare against the field scale of T-driven flow
    for f in ("u", "v"):
        a, b = g.fetch(f), o.fetch(f)
        assert np.abs(a - b).max() <= 1e-4 * max(np.abs(b).max(), 1e-12) + 1e-12, f


@pytest.mark.parametrize("iface", [0, 1])
def test_split_256_over_5000_steps(lf, ctx, iface):
    """256 x 256 split cavity, Ra 1e6, Pr 0.71, seeded T0 (uniform +-1e-6),
    5000 steps with each closure (non-equilibrium extrapolation, finite-
    difference gradients): the interface of Eq 91-95 exchanging every step
    while the boundary layers form.  FP64 within 1e-10 and FP32 within 1e-4
    of the oracle, element by element on u, v, T and rho, and the Nusselt
    numbers."""
    oracle.set_threads(16)
    n = 256
    T0 = perturbation(n, n, 1908083860)
    o = oracle.DDCase(n, n, oracle.SPLIT, iface).set_physics(1e6, 0.71).set_cavity_walls()
    o.init(T0)
    o.step(5000)
    no = o.nusselt()
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        print(f"split 256^2 iface {iface} {prec}: 5000 steps", flush=True)
        g = lf.Case(ctx, n, n, prec, mode=lf.MODE_SPLIT, iface=iface)
        g.set_physics(1e6, 0.71).set_cavity_walls().init(T0)
        assert abs(g.params()["nu"] - o.params["nu"]) < 1e-15
        g.step(5000)
        check(g, o, tol)
        ng = g.nusselt()
        for k in ("nu_hot", "nu_cold", "nu_hot_max"):
            assert abs(ng[k] - no[k]) <= tol * abs(no[k]), (prec, k)
        g.close()


@pytest.mark.parametrize("iface", [0, 1])
def test_split_full_size_200_steps(lf, ctx, iface):
    """4096 x 4096 split cavity, Ra 1e6, FP32, in the benchmark's launch
    configuration, 200 steps with each closure: element-wise parity with the
    oracle on u, v, T within 1e-4 of each field's maximum."""
    oracle.set_threads(16)
    n = 4096
    print(f"split 4096^2 iface {iface}: 200 steps", flush=True)
    g, o = pair(lf, ctx, n, n, "f32", iface, Ra=1e6, T0=perturbation(n, n, 1908083860))
    g.step(200)
    o.step(200)
    check(g, o, 1e-4, ("u", "v", "T"))


@pytest.mark.parametrize("iface", [0, 1])
def test_split_steady_state_parity(lf, ctx, iface):
    """64 x 64, Ra 1e4, FP64, both closures run to a 1e-9 residual (the
    level of Eq 93 gives the split mode a fixed point): the steady fields
    and Nusselt numbers against the oracle's own steady state."""
    oracle.set_threads(8)
    n = 64
    g = lf.Case(ctx, n, n, "f64", mode=lf.MODE_SPLIT, iface=iface).set_physics(1e4, 0.71)
    g.set_cavity_walls().init()
    sg, rg, _ = g.run_to_steady(tol=1e-9, check_every=1000, max_steps=80000)
    o = oracle.DDCase(n, n, oracle.SPLIT, iface).set_physics(1e4, 0.71).set_cavity_walls().init()
    so, ro = o.run_to_steady(tol=1e-9, check_every=1000, max_steps=80000)
    assert sg == so and max(rg) <= 1e-9 and ro.max() <= 1e-9, (sg, so, rg, ro)
    check(g, o, 1e-8)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= 1e-8 * abs(no[k]), (k, ng[k], no[k])


@pytest.mark.parametrize("iface", [0, 1])
def test_split_full_size_20000_steps(lf, ctx, iface):
    """The 4096 x 4096 split cavity of the benchmark (Ra 1e6, FP32) over
    20 000 steps with each closure: the fields stay finite, the LBM zone
    (nodes 0 .. ib) keeps its mass to 1e-6 of its 2050 x 4096 at init (the
    level of Eq 93), and the wall Nusselt numbers are finite and positive."""
    n = 4096
    g = lf.Case(ctx, n, n, "f32", mode=lf.MODE_SPLIT, iface=iface).set_physics(1e6, 0.71)
    g.set_cavity_walls().init(perturbation(n, n, 1908083860))
    m0 = g.mass()[0]
    assert abs(m0 - 2050 * 4096) < 1e-3
    g.step(20000)
    for f in ("u", "v", "T"):
        assert np.isfinite(g.fetch(f)).all(), f
    assert abs(g.mass()[0] - m0) < 1e-6 * m0
    nu = g.nusselt()
    for k in ("nu_hot", "nu_cold"):
        assert np.isfinite(nu[k]) and 0.0 < nu[k] < 100.0, (k, nu)


def pure_pair(lf, ctx, nx, ny, prec, mode, omode, Ra=1e5, Pr=0.71, T0=None, conv=0):
    g = lf.Case(ctx, nx, ny, prec, mode=mode)
    g.set_physics(Ra, Pr, conv=conv).set_cavity_walls().init(T0)
    o = oracle.DDCase(nx, ny, omode).set_physics(Ra, Pr).set_cavity_walls()
    o.set_lattice(o.params["nu"], o.params["alpha"], o.params["gbeta"], 0.0, conv=conv)
    o.init(T0)
    assert abs(g.params()["nu"] - o.params["nu"]) < 1e-15
    return g, o


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("nx,ny", [(40, 24), (203, 70)])
def test_pure_fv_parity(lf, ctx, prec, tol, nx, ny):
    """The FV-only cavity (the single FV method of Sec. 4.2) against the
    oracle: 40 x 24 runs on wall waves only; 203 x 70 also on the interior
    (direct-addressed) path, with ragged rows and columns."""
    oracle.set_threads(8)
    T0 = perturbation(nx, ny, 41, amp=0.1)
    g, o = pure_pair(lf, ctx, nx, ny, prec, lf.MODE_PURE_FV, oracle.PURE_FV, T0=T0)
    g.step(500)
    o.step(500)
    check(g, o, tol)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= tol * abs(no[k]), k


@pytest.mark.parametrize("conv", [1, 2])
def test_pure_fv_central_and_upwind(lf, ctx, conv):
    oracle.set_threads(8)
    nx, ny = 150, 40
    T0 = perturbation(nx, ny, 42, amp=0.1)
    g, o = pure_pair(lf, ctx, nx, ny, "f64", lf.MODE_PURE_FV, oracle.PURE_FV, T0=T0, conv=conv)
    g.step(300)
    o.step(300)
    check(g, o, 1e-10)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("nx,ny", [(40, 24), (130, 70)])
def test_pure_lbm_parity(lf, ctx, prec, tol, nx, ny):
    """The LBM-only cavity (D2Q9 flow + D2Q5 heat on the whole box, the single
    LBM method of Sec. 4.2) against the oracle."""
    oracle.set_threads(8)
    T0 = perturbation(nx, ny, 43, amp=0.1)
    g, o = pure_pair(lf, ctx, nx, ny, prec, lf.MODE_PURE_LBM, oracle.PURE_LBM, T0=T0)
    g.step(500)
    o.step(500)
    check(g, o, tol)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= tol * abs(no[k]), k


def test_pure_modes_conserve(lf, ctx):
    """Closed boxes: the LBM-only cavity keeps sum f to rounding; the FV-only
    cavity keeps its mean pressure (sum of 1 + 3 p) at its initial level."""
    n = 48
    T0 = perturbation(n, n, 44, amp=0.2)
    for mode in (lf.MODE_PURE_LBM, lf.MODE_PURE_FV):
        g = lf.Case(ctx, n, n, "f64", mode=mode).set_physics(1e5, 0.71).set_cavity_walls()
        g.init(T0)
        m0, _ = g.mass()
        g.step(700)
        m1, _ = g.mass()
        assert abs(m1 - m0) <= 1e-10 * n * n, (mode, m0, m1)


def test_pure_mode_errors(lf, ctx):
    for mode in (lf.MODE_PURE_FV, lf.MODE_PURE_LBM):
        g = lf.Case(ctx, 32, 32, mode=mode)
        with pytest.raises(lf.LFError) as e:
            g.set_wall(lf.W, lf.WALL_PERIODIC, 0.0, lf.T_PERIODIC, 0.0)
        assert e.value.status == lf.LF_ENOTIMPL
        with pytest.raises(lf.LFError) as e:  # only the north wall slides
            g.set_wall(lf.E, lf.WALL_NOSLIP, 0.05, lf.T_ADIABATIC, 0.0)
        assert e.value.status == lf.LF_ENOTIMPL
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 32, 32, mode=99)
    assert e.value.status == lf.LF_EINVAL


def h_pair(lf, ctx, nx, ny, prec, iface, Ra=1e5, Pr=0.71, T0=None):
    """The horizontally divided cavity (LBM below, FV above) through the
    library, and the oracle's vertically divided cavity stored transposed
    with gravity along -x."""
    g = lf.Case(ctx, nx, ny, prec, mode=lf.MODE_SPLIT_H, iface=iface)
    g.set_physics(Ra, Pr).set_cavity_walls().init(T0)
    p = g.params()
    o = oracle.DDCase(ny, nx, oracle.SPLIT, iface)
    o.set_lattice(p["nu"], p["alpha"], p["gbeta"], 0.0).set_gravity_axis("x")
    o.set_thermal(oracle.S, True, 0.5).set_thermal(oracle.N, True, -0.5)
    o.set_thermal(oracle.W, False).set_thermal(oracle.E, False)
    o.init(None if T0 is None else np.ascontiguousarray(T0.T))
    return g, o


def h_check(g, o, tol):
    pairs = (("u", "v"), ("v", "u"), ("T", "T"), ("rho", "rho"))
    errs = {}
    for fg, fo in pairs:
        a, b = g.fetch(fg), o.fetch(fo).T
        if fg == "rho":
            a, b = a - 1, b - 1
        errs[fg] = rel_linf(a, b)
    for f, e in errs.items():
        assert e <= tol, (f, e, errs)
    T = o.fetch("T").T
    ny = T.shape[0]
    hot = (2.0 * ny * (0.5 - T[:, 0])).mean()
    cold = (2.0 * ny * (T[:, -1] + 0.5)).mean()
    nu = g.nusselt()
    assert abs(nu["nu_hot"] - hot) <= tol * abs(hot) and abs(nu["nu_cold"] - cold) <= tol * abs(cold)


@pytest.mark.parametrize("iface", [0, 1])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_horizontal_division_parity(lf, ctx, iface, prec, tol):
    """Fig. 17b's division: 48 wide, 64 high, LBM rows 0..31 (+ overlap),
    FV above, against the oracle's transposed vertical division."""
    oracle.set_threads(8)
    nx, ny = 48, 64
    T0 = perturbation(nx, ny, 61, amp=0.1)
    g, o = h_pair(lf, ctx, nx, ny, prec, iface, T0=T0)
    g.step(600)
    o.step(600)
    h_check(g, o, tol)


def test_horizontal_division_ragged_fp64(lf, ctx):
    """77 wide, 138 high at Ra 1e6: ragged tiles in both stored directions."""
    oracle.set_threads(8)
    nx, ny = 77, 138
    T0 = perturbation(nx, ny, 62, amp=0.05)
    g, o = h_pair(lf, ctx, nx, ny, "f64", 0, Ra=1e6, T0=T0)
    g.step(500)
    o.step(500)
    h_check(g, o, 1e-10)
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 64, 65, mode=lf.MODE_SPLIT_H)  # odd divided extent
    assert e.value.status == lf.LF_EINVAL


@pytest.mark.parametrize("mode", ["split", "pure_fv"])
def test_pressure_fetch(lf, ctx, mode):
    """LF_FIELD_P: the kinematic pressure c_s^2 (rho - 1), which in the FV
    zone is its own p (the oracle's raw FV pressure) and in the LBM zone the
    lattice pressure; FP64, 64 x 48, 600 steps."""
    oracle.set_threads(8)
    nx, ny = 64, 48
    T0 = perturbation(nx, ny, 33, amp=0.1)
    gm, om = (lf.MODE_SPLIT, oracle.SPLIT) if mode == "split" else (lf.MODE_PURE_FV, oracle.PURE_FV)
    g = lf.Case(ctx, nx, ny, "f64", mode=gm).set_physics(1e5, 0.71).set_cavity_walls().init(T0)
    o = oracle.DDCase(nx, ny, om).set_physics(1e5, 0.71).set_cavity_walls().init(T0)
    g.step(600)
    o.step(600)
    p = g.fetch("p")
    ref = (o.fetch("rho") - 1.0) / 3.0
    assert np.abs(p - ref).max() <= 1e-10 * np.abs(ref).max()
    s = nx // 2
    raw = o.fetch("p")  # the FV cells' own pressure
    assert np.abs(p[:, s:] - raw[:, s:]).max() <= 1e-10 * np.abs(raw[:, s:]).max()
    assert np.abs(p - (g.fetch("rho") - 1.0) / 3.0).max() <= 1e-15
