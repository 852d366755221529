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


def _tone_fit(series, wt):
    """Least-squares amplitude F = a + ib of series ~ a cos(wt) + b sin(wt), per column."""
    basis = np.stack([np.cos(wt), np.sin(wt)], axis=1)
    coef, *_ = np.linalg.lstsq(basis, series.reshape(len(wt), -1), rcond=None)
    return (coef[0] + 1j * coef[1]).reshape(series.shape[1:])


def test_absorption_equals_flux_balance():
    """Discrete Poynting theorem.  In steady state with Ez = Re(F e^{-i w t}) at the
    half-integer times, eliminating H from eqs. 18-20 gives the five-point equation
    L F + q F = 0 with q = 2i s (e^{-i th} - Ce e^{i th}) / (S1 Cb), th = w dt / 2,
    s = sin th (normalised Cb = S1 / (eps_r (1 + a)), eq. 17 with a = n k w dt / eps_r).
    Summing F* (L F + q F) over the rows between the monitors leaves the Wronskian
    fluxes through the two bounding lines, so the power absorbed in the cells,
    sum Im(q) |F|^2, divided by the incident flux Nx |F_inc|^2 sin(ky_0 h), must equal
    1 - R - T from the monitors' Bloch orders (eqs. 31-34), and the flux through the
    transmission row must equal T.  q is built here from (n, k) and the label map,
    not from the oracle's coefficient tables."""
    nx, ny = 48, 192
    lab = _grating(nx=nx, ny=ny, seed=11)
    lab[150:] = 0                                   # vacuum from below the TF/SF line up
    nk = np.array([[1.0, 0.0], [1.5, 0.04], [1.3, 0.01]])
    prob = O.Problem(nx=nx, ny=ny, h=20e-9, lambda0=600e-9, n_steps=9000, n_pml=24)
    ce, cb = O.pixel_coefficients(prob, lab, nk)
    e_inc, h_inc = O.incident(prob)
    st, mon, _ = O.run(prob, ce, cb, e_inc, h_inc, n_end=prob.dft_start)
    hist = []
    for n0 in range(prob.dft_start, prob.n_steps, 750):
        n1 = min(prob.n_steps, n0 + 750)
        st, mon, h = O.run(prob, ce, cb, e_inc, h_inc, state=st, n_begin=n0, n_end=n1, mon=mon, history=True)
        hist.append(h)
    hist = np.concatenate(hist)
    R, T, A, _ = O.spectra(prob, mon, O.incident_sums(prob, e_inc))

    s1 = prob.courant / np.sqrt(2.0)
    wdt = 2.0 * np.pi * s1 * prob.h / prob.lambda0
    wt = wdt * (np.arange(prob.dft_start, prob.n_steps) + 0.5)
    F = _tone_fit(hist, wt)
    f_inc = _tone_fit(e_inc[prob.dft_start:, None], wt)[0]

    th, s = 0.5 * wdt, np.sin(0.5 * wdt)
    n, k = nk[lab, 0], nk[lab, 1]
    eps = n * n - k * k
    a = n * k * wdt / eps
    Ce, Cb = (1 - a) / (1 + a), s1 / (eps * (1 + a))
    q = 2j * s * (np.exp(-1j * th) - Ce * np.exp(1j * th)) / (s1 * Cb)

    ky0 = 2.0 * np.arcsin(s / s1)
    inc_flux = nx * abs(f_inc) ** 2 * np.sin(ky0)
    j0, j1 = prob.j_trn + 1, prob.j_src - 1
    absorbed = (q[j0:j1 + 1].imag * np.abs(F[j0:j1 + 1]) ** 2).sum() / inc_flux
    down = lambda j: -np.imag(np.conj(F[j]) * F[j + 1]).sum() / inc_flux
    assert A > 0.05
    assert absorbed == pytest.approx(A, abs=2e-5)
    assert down(j1) - down(j0 - 1) == pytest.approx(absorbed, abs=1e-6)   # Green's identity
    assert down(prob.j_trn) == pytest.approx(T, abs=2e-5)
    assert down(j1) == pytest.approx(1.0 - R, abs=2e-5)
