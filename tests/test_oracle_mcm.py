"""Pins of the Monte Carlo temperature oracle and the coupled LBM-MCM
reference (Sec. 6, Eq 97-102, Table 3)."""
import json
import os

import numpy as np

from oracle.mcm import MCMCase, exact_expectation, probabilities, walk

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_probabilities_sum_to_one_and_reduce_to_eq98():
    rng = np.random.default_rng(2)
    u, v = rng.uniform(-0.05, 0.05, (2, 50))
    P = probabilities(u, v, 0.08)
    assert np.abs(sum(P) - 1.0).max() < 1e-15
    assert min(p.min() for p in P) > 0.0
    assert all(abs(p - 0.25) < 1e-16 for p in probabilities(0.0, 0.0, 0.3))


def test_conduction_matches_eq112():
    """Fig. 40's square: the lid at theta = 1, the other walls at 0; the
    walkers' expectation against the series of Eq 112 at the cell centres,
    second order away from the lid's corner singularities."""
    n = 32
    z = np.zeros((n, n))
    T = exact_expectation(z, z, 0.1, [1, 1, 1, 1], [0.0, 0.0, 0.0, 1.0])
    X = (np.arange(n) + 0.5) / n
    Y = X[:, None]
    th = np.zeros((n, n))
    for k in range(1, 800):
        # sinh(k pi Y) / sinh(k pi), written without overflow
        r = np.exp(k * np.pi * (Y - 1)) * (1 - np.exp(-2 * k * np.pi * Y)) / (1 - np.exp(-2 * k * np.pi))
        th += 2 / np.pi * ((-1) ** (k + 1) + 1) / k * r * np.sin(k * np.pi * X[None, :])
    rows = (np.arange(n) + 0.5) / n < 0.8
    assert np.abs(T - th)[rows].max() < 2e-3
    assert np.abs(T - th).max() < 0.03


def test_walkers_estimate_the_linear_system():
    """Eq 101's walks (splitmix64 draws) from three nodes of a 10 x 10 box
    with a non-uniform velocity field: the mean recorded wall temperature
    lies within 4 standard errors of the exact expectation (Eq 97)."""
    n = 10
    J, I = np.mgrid[0:n, 0:n]
    u = 0.03 * np.sin(np.pi * (J + 0.5) / n)
    v = -0.02 * np.cos(np.pi * (I + 0.5) / n)
    tfix, Tw = [1, 1, 0, 0], [0.5, -0.5, 0.0, 0.0]
    al = 0.06
    T = exact_expectation(u, v, al, tfix, Tw)
    N = 1500
    for (i, j) in ((2, 3), (7, 5), (5, 9)):
        rec = [walk(i, j, w, N, 1908083867, u, v, al, tfix, Tw, 100000)[0] for w in range(N)]
        assert all(r is not None for r in rec)
        est = float(np.mean(rec))
        assert abs(est - T[j, i]) <= 4 * 0.5 / np.sqrt(N), (i, j, est, T[j, i])


def test_coupled_ra1e4_matches_table3():
    """Coupled LBM-MCM (the expectation of the walkers, S = 200) on 64 x 64
    at Ra 1e4: Nu_max within 3 % of Table 3's LBM-MCM and Ref [46] values,
    its height within 1.5 cells of 0.15, the hot-wall average within 3 % of
    Table 3's Nu_ave."""
    with open(os.path.join(HERE, "paper_tables.json")) as f:
        tab = json.load(f)
    c = MCMCase(64, 64, S=200).set_physics(1e4, 0.71).init()
    c.step(12000)
    nu = c.nusselt()
    for ref in (tab["table3_nu_max"]["lbm_mcm"]["1e4"], tab["table3_nu_max"]["reference_46"]["1e4"]):
        assert abs(nu["nu_hot_max"] - ref) / ref < 0.03, (nu, ref)
    assert abs(nu["y_hot_max"] - 0.15) * 64 <= 1.5
    ref = tab["table3_nu_avg"]["lbm_mcm"]["1e4"]
    assert abs(nu["nu_hot"] - ref) / ref < 0.03, (nu, ref)
