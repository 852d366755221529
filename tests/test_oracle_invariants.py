"""Oracle pins from invariants of the discrete method: energy balance of a
lossless grating with discrete-flux weights, empty-domain transmission and
absorbing-layer reflection, TF/SF leakage, periodic-shift and mirror
symmetry, and the CFL limit."""
import numpy as np
import pytest

import oracle as O


def _grating(nx=112, ny=256, seed=0):
    rng = np.random.default_rng(seed)
    lab = np.zeros((ny, nx), np.uint8)
    blk = rng.integers(0, 3, size=(10, -(-nx // 8)))
    lab[90:170] = np.kron(blk, np.ones((8, 8), np.uint8))[:80, :nx]
    return lab


@pytest.fixture(scope="module")
def lossless_grating():
    lab = _grating()
    nk = np.array([[1.0, 0.0], [1.5, 0.0], [1.3, 0.0]])
    prob = O.Problem(nx=112, ny=256, h=20e-9, lambda0=600e-9, n_steps=16000, n_pml=32)
    return prob, lab, nk, O.simulate(prob, lab, nk)


def test_lossless_grating_conserves_energy(lossless_grating):
    prob, lab, nk, r = lossless_grating
    o = r["orders"]
    assert (o["w"] > 0).sum() >= 5                     # several Bloch orders propagate
    assert abs(r["R"] + r["T"] - 1.0) < 2e-5
    # weights are sin(ky_m h)/sin(ky_0 h): <= 1, symmetric in m
    w = o["w"]
    assert w.max() == pytest.approx(1.0) and np.allclose(w, w[::-1][: len(w)] if len(w) % 2 else w)


def test_literal_unweighted_orders_break_energy_balance(lossless_grating):
    prob, lab, nk, r = lossless_grating
    p2 = O.Problem(**{**prob.__dict__, "literal_orders": 1})
    R, T, A, _ = O.spectra(p2, r["mon"], r["inc"])
    assert R + T - 1.0 > 0.05


def test_lossy_grating_absorbs():
    lab = _grating(nx=64, seed=3)
    nk = np.array([[1.0, 0.0], [1.5, 0.05], [1.3, 0.0]])
    prob = O.Problem(nx=64, ny=256, h=20e-9, lambda0=600e-9, n_steps=6000, n_pml=16)
    r = O.simulate(prob, lab, nk)
    assert 0.0 < r["R"] < 1.0 and 0.0 < r["T"] < 1.0 and r["A"] > 0.01


def test_empty_domain_transmits_and_layers_absorb():
    prob = O.Problem(nx=4, ny=256, h=20e-9, lambda0=600e-9, n_steps=3000, n_pml=16)
    r = O.simulate(prob, np.zeros((256, 4), np.uint8), np.array([[1.0, 0.0]]))
    # R of an empty domain is the absorbing layer's reflection: amplitude <= 1e-4
    assert np.sqrt(r["R"]) < 1e-4
    assert abs(r["T"] - 1.0) < 2e-5


def test_tfsf_line_does_not_leak():
    ny, nx = 256, 8
    prob = O.Problem(nx=nx, ny=ny, h=20e-9, lambda0=600e-9, n_steps=3000, n_pml=16)
    ce, cb = O.pixel_coefficients(prob, np.zeros((ny, nx), np.uint8), np.array([[1.0, 0.0]]))
    e_inc, h_inc = O.incident(prob)
    # (a) before anything returns from the 1D grid's own absorber (information moves one
    # cell per step), the scattered-field region holds roundoff only
    n_a = 2 * prob.aux_pad - 8
    st, _, _ = O.run(prob, ce, cb, e_inc, h_inc, n_end=n_a)
    sf = np.abs(st.ez[prob.j_src + 1:]).max()
    tf = np.abs(st.ez[: prob.j_src + 1]).max()
    assert tf > 0.05 and sf < 1e-13 * tf
    # (b) later, and before the 2D layers can echo, the leak is bounded by the 1D
    # absorber's own reflection
    n_b = 2 * (prob.j_src - prob.n_pml) - 20
    st, _, _ = O.run(prob, ce, cb, e_inc, h_inc, n_end=n_b)
    sf = np.abs(st.ez[prob.j_src + 1:]).max()
    tf = np.abs(st.ez[: prob.j_src + 1]).max()
    assert sf < 1e-7 * tf


def test_periodic_shift_invariance():
    lab = _grating(nx=64, seed=5)
    nk = np.array([[1.0, 0.0], [1.5, 0.03], [1.3, 0.01]])
    prob = O.Problem(nx=64, ny=256, h=20e-9, lambda0=600e-9, n_steps=2500, n_pml=16)
    a = O.simulate(prob, lab, nk)
    b = O.simulate(prob, np.roll(lab, 17, axis=1), nk)
    assert b["R"] == pytest.approx(a["R"], rel=1e-11, abs=1e-14)
    assert b["T"] == pytest.approx(a["T"], rel=1e-11, abs=1e-14)
    assert np.allclose(np.roll(a["state"].ez, 17, axis=1), b["state"].ez, rtol=1e-9, atol=1e-12 * np.abs(a["state"].ez).max())


def test_mirror_symmetry():
    half = _grating(nx=32, seed=7)
    lab = np.concatenate([half, half[:, ::-1]], axis=1)     # symmetric about x = Lx/2
    nk = np.array([[1.0, 0.0], [1.5, 0.03], [1.3, 0.01]])
    prob = O.Problem(nx=64, ny=256, h=20e-9, lambda0=450e-9, n_steps=2500, n_pml=16)
    r = O.simulate(prob, lab, nk)
    o = r["orders"]
    m = o["m"]
    for mm in range(1, 4):
        a = o["ref"][m == mm][0]
        b = o["ref"][m == -mm][0]
        assert a == pytest.approx(b, rel=1e-9, abs=1e-15)
    ez = r["state"].ez
    assert np.allclose(ez, ez[:, ::-1], rtol=1e-9, atol=1e-12 * np.abs(ez).max())


def test_courant_above_one_diverges():
    lab = _grating(nx=32, seed=1)
    nk = np.array([[1.0, 0.0], [1.5, 0.0], [1.3, 0.0]])
    grow = {}
    for S in (0.99, 1.05):
        prob = O.Problem(nx=32, ny=256, h=20e-9, lambda0=600e-9, n_steps=1500, n_pml=16, courant=S)
        r = O.simulate(prob, lab, nk)
        grow[S] = np.abs(r["state"].ez).max()
    assert grow[0.99] < 10.0
    assert not np.isfinite(grow[1.05]) or grow[1.05] > 1e6
