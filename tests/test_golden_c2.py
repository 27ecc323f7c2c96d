"""The stored 512 x 512 steady state (written by tests/golden/make_c2_steady.py
from the oracle) against what the paper prints: Table 1's maximum hot-wall
Nusselt number at Ra 1e6 within the paper's 3 % band, Table 2's location
within 1.5 cells, and the steady balance of the hot- and cold-wall fluxes."""
import json
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEYS = ("nu_hot", "nu_cold", "nu_hot_max", "y_hot_max", "nu_cold_max", "y_cold_max",
        "nu_hot_o2", "nu_cold_o2")


@pytest.fixture(scope="module")
def golden():
    p = os.path.join(HERE, "c2_steady_512.npz")
    if not os.path.exists(p):
        pytest.skip("golden steady state not generated")
    return np.load(p)


def test_stored_state_is_steady(golden):
    assert float(np.max(golden["residual"])) <= float(golden["tol"]) == 1e-8
    nu = dict(zip(KEYS, golden["nusselt"]))
    assert abs(nu["nu_hot"] - nu["nu_cold"]) <= 1e-5 * nu["nu_hot"]
    # centro-symmetry of the side-heated cavity: T(i, j) = -T(n-1-i, n-1-j)
    assert np.abs(golden["T_west"] + golden["T_east"][::-1]).max() <= 1e-5


def test_table1_table2_at_ra1e6(golden):
    with open(os.path.join(HERE, "paper_tables.json")) as f:
        tab = json.load(f)
    nu = dict(zip(KEYS, golden["nusselt"]))
    ref_max = tab["table1_nu_max"]["reference_41"]["1e6"]
    ref_y = tab["table2_y_of_nu_max"]["reference_41"]["1e6"]
    assert abs(nu["nu_hot_max"] - ref_max) / ref_max < 0.03, (nu["nu_hot_max"], ref_max)
    assert abs(nu["y_hot_max"] - ref_y) * 512 <= 1.5 + 0.5, (nu["y_hot_max"], ref_y)
    assert abs(nu["nu_hot_o2"] - nu["nu_hot"]) / nu["nu_hot"] < 0.01


def test_full_field_matches_the_fp64_samples(golden):
    """The stored FP32 full fields are the FP64 steady state rounded: on every
    4th node they equal the stored FP64 samples to FP32 rounding, their maxima
    are the stored maxima, and T is centro-symmetric over the whole field."""
    mx = golden["max_abs"]
    for k, name in enumerate(("u", "v", "T")):
        full = golden[name + "32"].astype(np.float64)
        assert full.shape == (512, 512)
        samp = golden[name + "_s"]
        assert np.abs(full[::4, ::4] - samp).max() <= 2.0 ** -24 * np.abs(samp).max(), name
        assert abs(np.abs(full).max() - mx[k]) <= 2.0 ** -24 * mx[k], name
    T = golden["T32"].astype(np.float64)
    assert np.abs(T + T[::-1, ::-1]).max() <= 1e-5
