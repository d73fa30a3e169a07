"""Scenario-geometry helpers against the worked numbers the paper prints
(fixture tests/golden/paper_worked_numbers.json; each entry names its passage)."""
import json
import os

import pytest

from paper_1905_05727_amd import scenario as S

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_worked_numbers.json")))


def test_regular_spacing_eq6_1():
    g = G["regular_spacing"]
    d = S.regular_spacing(g["d_c_m"], g["phi"])
    assert round(d * 1e3, 3) == pytest.approx(g["delta_c_m"] * 1e3, abs=1e-12)


@pytest.mark.parametrize("case", G["number_density_3d"]["cases"])
def test_number_density(case):
    rn = S.number_density_3d(case["phi"], case["d_c_m"]) * 1e-9   # per mm^3
    assert abs(rn - case["rho_N_per_mm3"]) <= 1.0


def test_min_vs_mean_spacing():
    g = G["spacing_comparison"]
    assert 2.5 * g["d_c_m"] == pytest.approx(g["min_spacing_m"], rel=1e-12)
    assert round(S.regular_spacing(g["d_c_m"], g["phi"]), 6) == pytest.approx(g["mean_spacing_m"])


@pytest.mark.parametrize("case", G["grid_points"]["cases"])
def test_grid_points(case):
    nx = round(case["L_m"] / case["dx_m"])
    ny = round(case["W_m"] / case["dx_m"])
    assert [nx, ny] == case["points"]


def test_cavity_count_eq7():
    """Eq. (7) for the random field of the paper (phi = 8 %, 24 x 2 mm): the
    count of 100 um cavities is 'hundreds' and close to 489."""
    n = S.cavity_count(0.08, 0.024, 0.002, 1e-4)
    assert 488 < n < 490


def test_regular_array_matches_paper_grid():
    """The regular array at 100 cells per diameter reproduces the paper's
    24000 x 313 grid (App. A) with the Eq. (6_1) spacing and porosity phi."""
    sc = S.regular_array()
    g = G["grid_points"]["cases"][0]["points"]
    assert [sc.nx, sc.ny] == g
    assert sc.bc[2:] == ("periodic", "periodic")
    b = sc.meta["bubbles"]
    assert abs(b[1, 0] - b[0, 0] - S.regular_spacing(100.0, 0.08)) < 1e-9
    por = (sc.prim[0][:, 500:] > 0.5).mean()
    assert abs(por - 0.08) < 0.002
    import numpy as np
    assert np.array_equal(sc.prim, sc.prim[:, ::-1, :])      # mirror symmetric about mid-width


def test_random_cavities_follow_eq7_and_min_spacing():
    import numpy as np
    sc = S.random_cavities(length=6000, width=2000, seed=3)
    n = S.cavity_count(0.08, 5500.0, 2000.0, 100.0)
    assert sc.meta["ncavities"] == round(n)
    b = sc.meta["bubbles"]
    dx = b[:, 0][:, None] - b[:, 0][None, :]
    dy = np.abs(b[:, 1][:, None] - b[:, 1][None, :])
    dy = np.minimum(dy, 2000 - dy)                          # periodic across top/bottom
    d = np.sqrt(dx ** 2 + dy ** 2) + np.eye(len(b)) * 1e9
    assert d.min() >= 250.0                                 # 2.5 d_c (Sec. 3)
    assert abs((sc.prim[0][:, 500:] > 0.5).mean() - 0.08) < 0.005
