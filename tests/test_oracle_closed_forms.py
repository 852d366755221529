"""Oracle pins from printed numbers and closed forms: the CFL time step
(Sec. 2.3, checked against the paper's printed time steps of Sec. 3 and 4),
the material map of eqs. 1-2 and the loss coefficients of eq. 17."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def _round_sig(x, d):
    return float("%.*g" % (d, x))


@pytest.mark.parametrize("key", ["validation_grid", "dicot_mesh", "monocot_mesh"])
def test_time_step_matches_printed(key):
    g = GOLD[key]
    # the paper evaluates dt = h/(c sqrt 2) with c = 3e8; the oracle uses SI c
    dt = O.time_step(g["h_m"], g["courant"]) * O.C0 / g["c_used"]
    assert _round_sig(dt, g["digits"]) == pytest.approx(g["dt_s"], rel=1e-12)


def test_time_step_is_cfl_bound():
    h = 17e-9
    dt = O.time_step(h, 1.0)
    assert dt == pytest.approx(1.0 / (O.C0 * math.sqrt(2.0 / h ** 2)), rel=1e-15)
    assert O.time_step(h, 0.99) == pytest.approx(0.99 * dt, rel=1e-15)


def test_dicot_mesh_arithmetic():
    g = GOLD["dicot_mesh"]
    assert g["lambda0_min_m"] / g["n_cell_wall"] == pytest.approx(g["lambda_min_m"], rel=1e-5)
    dt = O.time_step(g["h_m"], 1.0) * O.C0 / g["c_used"]
    dur = g["n_steps"] * dt
    assert dur == pytest.approx(g["duration_s"], rel=0.02)
    assert round(dur / (400e-9 / g["c_used"])) == pytest.approx(g["periods_400nm"], abs=2)
    assert round(dur / (2500e-9 / g["c_used"])) == pytest.approx(g["periods_2500nm"], abs=1)


def test_material_vacuum_and_lossless():
    dt = O.time_step(20e-9, 0.99)
    w = 2 * math.pi * O.C0 / 600e-9
    eps, sig, ce, cb = O.material(1.0, 0.0, w, dt)
    assert (eps, sig, ce) == (1.0, 0.0, 1.0)
    assert cb == pytest.approx(dt / O.EPS0, rel=1e-15)
    eps, sig, ce, cb = O.material(1.52, 0.0, w, dt)
    assert ce == 1.0 and eps == pytest.approx(1.52 ** 2)
    assert cb == pytest.approx(dt / (O.EPS0 * 1.52 ** 2), rel=1e-15)


def test_material_lossy_closed_forms():
    dt = O.time_step(25e-9, 0.99)
    w = 2 * math.pi * O.C0 / 550e-9
    for n, k in [(1.45, 0.01), (1.7, 0.3), (1.36, 0.02), (2.0, 0.5)]:
        eps, sig, ce, cb = O.material(n, k, w, dt)
        assert eps == pytest.approx(n * n - k * k, rel=1e-15)          # eq. 1
        assert sig == pytest.approx(2 * w * O.EPS0 * n * k, rel=1e-15)  # eq. 2
        a = n * k * w * dt / eps                                       # sigma dt / (2 eps0 eps_r)
        assert ce == pytest.approx((1 - a) / (1 + a), rel=1e-14)       # eq. 17
        assert cb == pytest.approx(dt / (O.EPS0 * eps) / (1 + a), rel=1e-14)
        # the semi-implicit decay factor tracks exp(-sigma dt/(eps0 eps_r)) to third order
        assert abs(ce - math.exp(-2 * a)) <= 2 * a ** 3 + 1e-15


def test_cpml_profiles_shape():
    p = O.Problem(nx=4, ny=100, h=20e-9, lambda0=600e-9, n_steps=10, n_pml=16)
    pe, ph = O.cpml_profiles(p)
    inner = slice(17, 83)
    assert np.all(pe[inner, 1] == 0) and np.all(pe[inner, 2] == 1)
    # c < 0 and |c| grows towards the outer walls; b in (0, 1)
    assert np.all(pe[:16, 1] < 0) and np.all(pe[84:, 1] < 0)
    assert np.all(np.diff(np.abs(pe[:16, 1])) < 0)
    assert np.all((pe[:16, 0] > 0) & (pe[:16, 0] < 1))
    # symmetric grading top/bottom at each field's own position
    assert np.allclose(pe[:16, :], pe[::-1][:16, :], rtol=1e-12)
    assert np.allclose(ph[1:16], ph[::-1][:15], rtol=1e-12)
