"""GPU parity of the fused Mode H step against the FP64 oracle.

Every case runs the same seeded inputs through the C-ABI library (on the GPU)
and through the oracle (on the CPU) and compares element by element:
FP64 within 1e-10 relative L-infinity, FP32 within 1e-4 (the stated bar for
u, v, T and Nu).  Sizes span several 62-column strips and bands with ragged
edges; walls cover fixed/adiabatic temperature, sliding and periodic sides.
"""
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


def make_pair(lf, ctx, nx, ny, prec, *, physics=None, lattice=None, walls="cavity", T0=None,
              u0=None, v0=None):
    g = lf.Case(ctx, nx, ny, prec)
    o = oracle.Case(nx, ny)
    if physics is not None:
        g.set_physics(*physics)
        o.set_physics(*physics)
    else:
        g.set_lattice(*lattice)
        o.set_lattice(*lattice)
    if walls == "cavity":
        g.set_cavity_walls()
        o.set_cavity_walls()
    else:
        for side, (vel, uw, th, tw) in walls.items():
            g.set_wall(side, vel, uw, th, tw)
            o.set_wall(side, vel, uw, th, tw)
    g.init(T0, u0, v0)
    o.init(T0, u0, v0)
    return g, o


def compare(g, o, tol, fields=("u", "v", "T")):
    errs = {f: rel_linf(g.fetch(f), o.fetch(f)) for f in fields}
    for f, e in errs.items():
        assert e <= tol, (f, e, errs)
    return errs


def test_c1_fp64_10000_steps(lf, ctx):
    """64x64, Ra 1e4, Pr 0.71, U_char 0.1, FP64, 10,000 steps."""
    oracle.set_threads(8)
    g, o = make_pair(lf, ctx, 64, 64, "f64", physics=(1e4, 0.71))
    g.step(10000)
    o.step(10000)
    compare(g, o, 1e-10, ("u", "v", "T", "rho"))
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max", "nu_hot_o2", "nu_cold_o2"):
        assert abs(ng[k] - no[k]) <= 1e-10 * abs(no[k]), k
    assert ng["y_hot_max"] == no["y_hot_max"]


def test_c1_fp32_10000_steps(lf, ctx):
    g, o = make_pair(lf, ctx, 64, 64, "f32", physics=(1e4, 0.71))
    g.step(10000)
    o.step(10000)
    compare(g, o, 1e-4)
    ng, no = g.nusselt(), o.nusselt()
    for k in ("nu_hot", "nu_cold", "nu_hot_max"):
        assert abs(ng[k] - no[k]) <= 1e-4 * abs(no[k]), k


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
@pytest.mark.parametrize("band", [1, 5, 64])
def test_ragged_tiles_sliding_walls(lf, ctx, prec, tol, band):
    """200 x 77: three full 62-column strips plus a ragged one, ragged bands;
    asymmetric T0, a sliding north wall and a sliding west wall."""
    ctx.set_band(band)
    try:
        nx, ny = 200, 77
        T0 = perturbation(nx, ny, 5, amp=0.3)
        walls = {lf.W: (0, 0.0, 0, 0.5), lf.E: (0, 0.0, 0, -0.5),
                 lf.S: (0, 0.0, 1, 0.0), lf.N: (0, 0.03, 1, 0.0)}
        walls[lf.W] = (0, -0.01, 0, 0.5)
        g, o = make_pair(lf, ctx, nx, ny, prec, lattice=(0.04, 0.03, 2e-4, 0.0), walls=walls,
                         T0=T0)
        g.step(300)
        o.step(300)
        compare(g, o, tol, ("u", "v", "T", "rho"))
    finally:
        ctx.set_band(0)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_periodic_x_dirichlet_y(lf, ctx, prec, tol):
    """Periodic along x (wrap across strips), heated from below (Rayleigh-Benard-like)."""
    nx, ny = 130, 40
    walls = {lf.W: (1, 0, 2, 0), lf.E: (1, 0, 2, 0),
             lf.S: (0, 0.0, 0, 0.5), lf.N: (0, 0.0, 0, -0.5)}
    T0 = perturbation(nx, ny, 9, amp=0.05)
    g, o = make_pair(lf, ctx, nx, ny, prec, lattice=(0.05, 0.05, 5e-4, 0.0, 1e-6, 0.0),
                     walls=walls, T0=T0)
    g.step(400)
    o.step(400)
    compare(g, o, tol, ("u", "v", "T"))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_periodic_y_side_walls(lf, ctx, prec, tol):
    """A vertical slot: periodic along y, hot west and cold east walls, so
    the side-wall march serves the rows away from the seam and the general
    march the rows that wrap."""
    nx, ny = 130, 40
    walls = {lf.W: (0, 0.0, 0, 0.5), lf.E: (0, 0.0, 0, -0.5),
             lf.S: (1, 0, 2, 0), lf.N: (1, 0, 2, 0)}
    T0 = perturbation(nx, ny, 14, amp=0.05)
    g, o = make_pair(lf, ctx, nx, ny, prec, lattice=(0.05, 0.05, 5e-4, 0.0), walls=walls, T0=T0)
    g.step(400)
    o.step(400)
    compare(g, o, tol, ("v", "T"))
    # the flow is vertical: u is measured against the slot's velocity scale
    vs = np.abs(o.fetch("v")).max()
    assert np.abs(g.fetch("u") - o.fetch("u")).max() <= tol * vs


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 2e-6)])
@pytest.mark.parametrize("axis,U", [("x", 0.05), ("x", -0.05), ("y", 0.04), ("y", -0.04)])
def test_quick_wall_ghost_closed_form(lf, ctx, prec, tol, axis, U):
    """QUICK's upstream ghost 2 T_w - T_edge beyond a fixed-temperature wall,
    against the closed form it must reproduce: for a temperature linear
    across the walls every face carries the exact value of the profile, so
    one step changes each cell by minus the divergence of u_f T(x_f) of the
    step's own velocities (the diffusive fluxes cancel).  130 cells across
    the walls: the wall strips' interior march and the general march (rows
    at the periodic seam) both take the ghost; tolerances absolute (T is
    0.1 .. 2.7)."""
    a, b, nw, npd = 0.1, 0.02, 130, 40
    nx, ny = (nw, npd) if axis == "x" else (npd, nw)
    g = lf.Case(ctx, nx, ny, prec).set_lattice(0.1, 0.07, 0.0)
    lo, hi = (lf.W, lf.E) if axis == "x" else (lf.S, lf.N)
    for sd in ((lf.S, lf.N) if axis == "x" else (lf.W, lf.E)):
        g.set_wall(sd, 1, 0.0, 2, 0.0)
    g.set_wall(lo, 0, 0.0, 0, a)
    g.set_wall(hi, 0, 0.0, 0, a + b * nw)
    prof = a + b * (np.arange(nw) + 0.5)
    T0 = np.tile(prof, (ny, 1)) if axis == "x" else np.tile(prof[:, None], (1, nx))
    vel0 = np.full((ny, nx), U)
    zero = np.zeros((ny, nx))
    g.init(T0, vel0 if axis == "x" else zero, zero if axis == "x" else vel0)
    g.step(1)
    vel = g.fetch("u" if axis == "x" else "v")
    T1 = g.fetch("T")
    Tface = a + b * np.arange(nw + 1)
    T0a, vela, T1a = (T0, vel, T1) if axis == "x" else (T0.T, vel.T, T1.T)
    uf = np.zeros((T0a.shape[0], nw + 1))
    uf[:, 1:-1] = 0.5 * (vela[:, :-1] + vela[:, 1:])
    F = uf * Tface[None, :]
    exp = T0a - (F[:, 1:] - F[:, :-1])
    assert (uf[:, 1].min() > 1e-3) if U > 0 else (uf[:, -2].max() < -1e-3)
    assert np.abs(T1a - exp).max() <= tol


@pytest.mark.parametrize("conv", [1, 2])
def test_central_and_upwind_convection(lf, ctx, conv):
    nx, ny = 70, 66
    T0 = perturbation(nx, ny, 13, amp=0.2)
    g, o = make_pair(lf, ctx, nx, ny, "f64", lattice=(0.05, 0.08, 3e-4, 0.0, 0.0, 0.0, conv),
                     T0=T0)
    g.step(200)
    o.step(200)
    compare(g, o, 1e-10)


def test_fully_periodic_uniform_flow(lf, ctx):
    """Uniform flow in a periodic box: the FV Fourier mode case of the oracle pins."""
    n = 96
    walls = {s: (1, 0, 2, 0) for s in (lf.W, lf.E, lf.S, lf.N)}
    jj, ii = np.mgrid[0:n, 0:n].astype(float)
    T0 = 0.3 * np.cos(2 * np.pi * (3 * ii - 2 * jj) / n)
    g, o = make_pair(lf, ctx, n, n, "f64", lattice=(0.1, 0.07, 0.0), walls=walls, T0=T0,
                     u0=np.full((n, n), 0.06), v0=np.full((n, n), -0.025))
    g.step(50)
    o.step(50)
    compare(g, o, 1e-11, ("T",))


def test_minimum_grid(lf, ctx):
    g, o = make_pair(lf, ctx, 8, 8, "f64", physics=(1e3, 0.71))
    g.step(500)
    o.step(500)
    compare(g, o, 1e-10)


def test_residual_mass_and_energy(lf, ctx):
    nx, ny = 96, 80
    T0 = perturbation(nx, ny, 21, amp=0.25)
    g, o = make_pair(lf, ctx, nx, ny, "f64", physics=(1e5, 0.71), T0=T0)
    for _ in range(3):
        g.step(250)
        o.step(250)
        rg, ro = g.residual(), o.residual()
        np.testing.assert_allclose(rg, ro, rtol=1e-9)
    mg, mo = g.mass(), o.mass()
    assert abs(mg[0] - mo[0]) <= 1e-12 * mo[0]
    assert abs(mg[0] - nx * ny) <= 1e-9 * nx * ny  # sum f conserved
    # adiabatic box: sum T conserved
    walls = {s: (0, 0.0, 1, 0.0) for s in (lf.W, lf.E, lf.S, lf.N)}
    g2, _ = make_pair(lf, ctx, nx, ny, "f32", lattice=(0.05, 0.05, 2e-3, 0.0), walls=walls, T0=T0)
    s0 = g2.mass()[1]
    g2.step(2000)
    s1 = g2.mass()[1]
    assert abs(s1 - s0) <= 1e-4 * np.abs(T0).sum()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_adiabatic_sliding_side_walls(lf, ctx, prec, tol):
    """140 x 50: the west wall adiabatic and sliding along +y, the east wall
    fixed, heated from below: the strips that hold a side wall (rows clear
    of the south and north walls) take the side-wall march."""
    nx, ny = 140, 50
    T0 = perturbation(nx, ny, 11, amp=0.2)
    walls = {lf.W: (0, 0.02, 1, 0.0), lf.E: (0, 0.0, 0, -0.5),
             lf.S: (0, 0.0, 0, 0.5), lf.N: (0, 0.0, 1, 0.0)}
    g, o = make_pair(lf, ctx, nx, ny, prec, lattice=(0.05, 0.04, 3e-4, 0.0), walls=walls, T0=T0)
    g.step(300)
    o.step(300)
    compare(g, o, tol, ("u", "v", "T", "rho"))


@pytest.mark.parametrize("nx", [184, 185])
def test_side_wall_strip_limits(lf, ctx, nx):
    """The east strip takes the side-wall march while the wall column is at
    most lane 60 (nx = 184: lane 60) and the general march past it
    (nx = 185: lane 61); FP64 against the oracle."""
    ny = 40
    T0 = perturbation(nx, ny, 13, amp=0.2)
    g, o = make_pair(lf, ctx, nx, ny, "f64", physics=(1e5, 0.71), T0=T0)
    g.step(200)
    o.step(200)
    compare(g, o, 1e-10, ("u", "v", "T", "rho"))


def test_band_invariance_bitwise_side_walls(lf, ctx):
    """An adiabatic east wall sliding along -y: bands of 1, 3 and 16 rows
    cut the side-wall strips differently (side-wall or general march for
    the same node) and give identical bits."""
    nx, ny = 150, 60
    T0 = perturbation(nx, ny, 12, amp=0.2)
    outs = []
    for band in (1, 3, 16):
        ctx.set_band(band)
        g = lf.Case(ctx, nx, ny, "f32").set_physics(1e5, 0.71).set_cavity_walls()
        g.set_wall(lf.E, lf.WALL_NOSLIP, -0.02, lf.T_ADIABATIC, 0.0).init(T0)
        g.step(150)
        outs.append([g.fetch(f) for f in ("u", "v", "T")])
    ctx.set_band(0)
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_band_invariance_bitwise(lf, ctx):
    """The step has no cross-node reduction: any band height gives identical bits."""
    nx, ny = 150, 90
    T0 = perturbation(nx, ny, 3, amp=0.2)
    outs = []
    for band in (1, 7, 32):
        ctx.set_band(band)
        g = lf.Case(ctx, nx, ny, "f32").set_physics(1e5, 0.71).set_cavity_walls().init(T0)
        g.step(120)
        outs.append([g.fetch(f) for f in ("u", "v", "T")])
    ctx.set_band(0)
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


def test_errors(lf, ctx):
    g = lf.Case(ctx, 16, 16, "f32")
    with pytest.raises(lf.LFError) as e:
        g.step(1)
    assert e.value.status == lf.LF_ESTATE
    with pytest.raises(lf.LFError) as e:
        g.set_lattice(0.0001, 0.1)  # tau too close to 1/2
    assert e.value.status == lf.LF_EUNSTABLE
    with pytest.raises(lf.LFError) as e:
        g.set_lattice(0.1, 0.3)  # explicit diffusion limit
    assert e.value.status == lf.LF_EUNSTABLE
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 4, 16)
    assert e.value.status == lf.LF_EINVAL
    # nine FP64 planes of 8192^2 exceed the step kernels' 32-bit byte range
    with pytest.raises(lf.LFError) as e:
        lf.Case(ctx, 8192, 8192, "f64")
    assert e.value.status == lf.LF_EINVAL
    # NaN input is reported by the residual
    g.set_lattice(0.1, 0.1).set_cavity_walls()
    T0 = np.zeros((16, 16))
    T0[3, 4] = np.nan
    g.init(T0).step(2)
    with pytest.raises(lf.LFError) as e:
        g.residual()
    assert e.value.status == lf.LF_EDIVERGED


def test_c2_size_500_steps_fp32(lf, ctx):
    """512 x 512, Ra 1e6 (the benchmark cavity) in the launch configuration the
    benchmark times: element-wise parity after 500 steps."""
    oracle.set_threads(8)
    n = 512
    T0 = perturbation(n, n, 1908083860)
    g, o = make_pair(lf, ctx, n, n, "f32", physics=(1e6, 0.71), T0=T0)
    g.step(500)
    o.step(500)
    compare(g, o, 1e-4)


def test_full_size_4096_in_bench_configuration(lf, ctx):
    """4096 x 4096, Ra 1e6, FP32 (the HBM-bound size the benchmark also times),
    with the automatic band height (4 rows, alternating march directions):
    element-wise parity with the oracle over the first 40 steps.  Velocities
    start from rest, so u and v are compared against the oracle's field scale
    plus a floor."""
    oracle.set_threads(16)
    n = 4096
    T0 = perturbation(n, n, 1908083860)
    g, o = make_pair(lf, ctx, n, n, "f32", physics=(1e6, 0.71), T0=T0)
    g.step(40)
    o.step(40)
    compare(g, o, 1e-4, ("T",))
    for f in ("u", "v"):
        a, b = g.fetch(f), o.fetch(f)
        assert np.abs(a - b).max() <= 1e-4 * max(np.abs(b).max(), 1e-12) + 1e-12, f
