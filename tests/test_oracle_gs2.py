"""Pins of the grid-setting-2 oracle (coarse FV temperature under the
lattice, one implicit energy step per S lattice steps, Sec. 5.1)."""
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.gs2 import SE, SN, SS, SW, GS2Case, quick_face, thomas

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_thomas_matches_a_dense_solve():
    rng = np.random.default_rng(11)
    n = 17
    lo, up = rng.uniform(-1, 0, (3, n)), rng.uniform(-1, 0, (3, n))
    di = 3 + rng.uniform(0, 1, (3, n))
    r = rng.normal(size=(3, n))
    x = thomas(lo, di, up, r)
    for k in range(3):
        A = np.diag(di[k]) + np.diag(lo[k, 1:], -1) + np.diag(up[k, :-1], 1)
        assert np.abs(x[k] - np.linalg.solve(A, r[k])).max() < 1e-13


def test_quick_is_exact_for_quadratics():
    # face at x = 0 between cells centred at -1/2 and +1/2 (unit cells)
    f = lambda x: 0.3 + 1.7 * x - 2.2 * x * x  # noqa: E731
    for w in (1.0, -1.0):
        v = quick_face(np.array(w), f(-1.5), f(-0.5), f(0.5), f(1.5))
        assert abs(float(v) - f(0.0)) < 1e-15


def test_interpolation_reproduces_fields_linear_in_x():
    c = GS2Case(20, 12).set_lattice(0.05, 0.1, 0.0)
    a, b = 0.2, -0.03  # T = a + b x on [0, 20]
    c.set_thermal(SW, True, a).set_thermal(SE, True, a + b * 20)
    X = 2.0 * np.arange(10) + 1.0
    Tc = np.tile(a + b * X, (6, 1))
    Tf = c.interp(Tc)
    x = np.arange(20) + 0.5
    assert np.abs(Tf - (a + b * x)[None, :]).max() < 1e-15


def test_conduction_limit_is_exact():
    """g beta = 0: the coarse T converges to the linear profile and the
    Nusselt number to 1/A exactly (one half-cell wall gradient per side)."""
    c = GS2Case(32, 16).set_lattice(0.05, 0.1, 0.0).init()
    c.step(32 * 300)
    lin = 0.5 - (np.arange(16) + 0.5) / 16
    assert np.abs(c.T - lin[None, :]).max() < 1e-13
    assert np.abs(c.Tf - (0.5 - (np.arange(32) + 0.5) / 32)[None, :]).max() < 1e-13
    assert abs(c.nusselt()["nu_hot"] - 0.5) < 1e-12
    assert np.abs(c.ux).max() == 0.0


def synthetic_step(seed):
    """A closed adiabatic box, a discretely divergence-free face velocity
    field from a stream function on the coarse cell corners, and a random T."""
    c = GS2Case(24, 24, S=7).set_lattice(0.05, 0.08, 0.0)
    for s in (SW, SE, SS, SN):
        c.set_thermal(s, False)
    rng = np.random.default_rng(seed)
    NX = NY = 12
    psi = np.zeros((NY + 1, NX + 1))
    psi[1:-1, 1:-1] = rng.uniform(-0.1, 0.1, (NY - 1, NX - 1))  # psi = 0 on the walls
    U = (psi[1:, :] - psi[:-1, :]) / 2.0    # u = d psi / dy on x-faces
    V = -(psi[:, 1:] - psi[:, :-1]) / 2.0   # v = -d psi / dx on y-faces
    T = rng.uniform(-0.5, 0.5, (NY, NX))
    return c, U, V, T


def test_energy_step_conserves_and_adi_reaches_the_direct_solve():
    c, U, V, T = synthetic_step(3)
    coef = c.assemble(U, V, T)
    aP, aW, aE, aS, aN, b = coef
    n = T.size
    idx = np.arange(n).reshape(T.shape)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [aP.ravel()]
    for a, dj, di in ((aW, 0, -1), (aE, 0, 1), (aS, -1, 0), (aN, 1, 0)):
        J, I = np.nonzero(a)
        rows.append(idx[J, I]); cols.append(idx[J + dj, I + di]); vals.append(-a[J, I])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), (n, n))
    direct = spla.spsolve(A.tocsc(), b.ravel()).reshape(T.shape)
    X = c.adi(coef, T.copy(), 400)
    assert np.abs(X - direct).max() < 1e-12
    # closed adiabatic box, divergence-free faces: sum T is kept
    assert abs(direct.sum() - T.sum()) < 1e-12 * np.abs(T).sum()
    # a uniform field stays uniform
    c2, U2, V2, _ = synthetic_step(4)
    Tu = np.full((12, 12), 0.37)
    Xu = c2.adi(c2.assemble(U2, V2, Tu), Tu.copy(), 5)
    assert np.abs(Xu - 0.37).max() < 1e-14


def test_table1_table2_at_ra1e4():
    """64 x 64 lattice, 32 x 32 temperature grid, Ra 1e4, Pr 0.71, S = 2NX:
    Nu_max within 3 % of Table 1 (this method and Ref [41]), its height
    within 1.5 lattice cells of Table 2, hot and cold walls balanced."""
    with open(os.path.join(HERE, "paper_tables.json")) as f:
        tab = json.load(f)
    c = GS2Case(64, 64).set_physics(1e4, 0.71).init()
    c.step(64 * 300)
    nu = c.nusselt()
    for ref in (tab["table1_nu_max"]["hybrid"]["1e4"], tab["table1_nu_max"]["reference_41"]["1e4"]):
        assert abs(nu["nu_hot_max"] - ref) / ref < 0.03, (nu, ref)
    y_ref = tab["table2_y_of_nu_max"]["hybrid"]["1e4"]
    assert abs(nu["y_hot_max"] - y_ref) * 64 <= 1.5, (nu, y_ref)
    assert abs(nu["nu_hot"] - nu["nu_cold"]) <= 1e-6 * nu["nu_hot"]
