"""The oracle against the numbers the paper prints for the side-heated cavity.

Table 1 (maximum hot-wall Nusselt number) and Table 2 (its location) of
Sec. 5.2, and the average Nusselt number of the benchmark column of Table 3
(Sec. 6.3.2); the paper states that all its methods are within 3 % of the
benchmark (Sec. 5.2).  The oracle is run to steady state on grids small
enough for the CPU suite; the 3 % band and a 1.5-cell band on the location
absorb the discretisation error of these grids.
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _tables():
    with open(GOLD) as f:
        return json.load(f)


def _steady(n, Ra, tol=1e-8):
    c = oracle.Case(n, n).set_physics(Ra, 0.71).set_cavity_walls().init()
    steps, r = c.run_to_steady(tol=tol, check_every=1000, max_steps=3_000_000)
    assert r.max() <= tol, r
    return c.nusselt(), steps


def _check(nu, n, ra_key, tab):
    ref_max = tab["table1_nu_max"]["reference_41"][ra_key]
    ref_y = tab["table2_y_of_nu_max"]["reference_41"][ra_key]
    assert abs(nu["nu_hot_o2"] - nu["nu_hot"]) / nu["nu_hot"] < 0.01
    # the second-order wall gradient is the quantity the benchmarks tabulate
    nu_max = max(nu["nu_hot_max"], 0)  # conservative half-cell flux
    assert abs(nu_max - ref_max) / ref_max < 0.03, (nu_max, ref_max)
    assert abs(nu["y_hot_max"] - ref_y) * n <= 1.5, (nu["y_hot_max"], ref_y)
    avg = tab["table3_nu_avg"]["reference_46"].get(ra_key)
    if avg is not None:
        assert abs(nu["nu_hot"] - avg) / avg < 0.03, (nu["nu_hot"], avg)


def test_ra1e4_table1_table2_table3():
    tab = _tables()
    oracle.set_threads(os.cpu_count() or 1)
    nu, _ = _steady(64, 1e4)
    _check(nu, 64, "1e4", tab)


def test_ra1e5_table1_table2_table3():
    tab = _tables()
    oracle.set_threads(os.cpu_count() or 1)
    nu, _ = _steady(96, 1e5)
    _check(nu, 96, "1e5", tab)


@pytest.mark.slow
def test_ra1e6_table1_table2():
    tab = _tables()
    oracle.set_threads(os.cpu_count() or 1)
    nu, _ = _steady(160, 1e6)
    _check(nu, 160, "1e6", tab)


def test_grid_convergence_of_average_nusselt():
    # Ra 1e4, diffusive scaling (nu, alpha fixed as the grid is refined):
    # the observed order of Nu_avg between n = 16, 32, 64 is about two
    oracle.set_threads(os.cpu_count() or 1)
    vals = []
    for n in (16, 32, 64):
        U = 0.1 * 16 / n
        c = oracle.Case(n, n).set_physics(1e4, 0.71, U_char=U).set_cavity_walls().init()
        _, r = c.run_to_steady(tol=1e-9, check_every=1000, max_steps=400_000)
        assert r.max() <= 1e-9
        vals.append(c.nusselt()["nu_hot"])
    p = np.log2(abs(vals[0] - vals[1]) / abs(vals[1] - vals[2]))
    assert 1.5 <= p <= 2.5, (vals, p)
