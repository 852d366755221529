"""Pins of the oracle's dispersive (Lorentz-Drude ADE) broadband path, Sec. 2.2:

* the discrete susceptibility of the polarisation recursion, built from the
  oracle's coefficients, tends to the continuous Lorentz and Drude forms as dt
  goes to 0, at second order;
* a pulsed run of a dispersive slab equals, at every monitor wavelength, the
  exact steady state of the discrete scheme (transfer matrix with the
  recursion's response);
* with no poles, the pulsed run equals monochromatic runs of the pinned CW path
  at each wavelength;
* a lossless dispersive grating conserves energy at every wavelength (several
  propagating orders);
* refined grids approach the continuous Fresnel/Fabry-Perot slab with the
  Lorentz permittivity at second order."""
import numpy as np
import pytest

import oracle as O
import closed_forms as CF

C0 = O.C0


def pulse_for(lams):
    """A Gaussian pulse covering the band to exp(-3) of its peak."""
    wlo, whi = 2 * np.pi * C0 / max(lams), 2 * np.pi * C0 / min(lams)
    w0 = 0.5 * (wlo + whi)
    tau = 4 * np.sqrt(3) / (whi - wlo)
    return 2 * np.pi * C0 / w0, tau, 4 * tau


def lorentz(eps_inf, d_eps, lam_p, gamma_rel, sigma=0.0):
    wp = 2 * np.pi * C0 / lam_p
    return [eps_inf, sigma, d_eps * wp * wp, wp, gamma_rel * wp]


def slab_problem(ny, h, lams, steps, n_pml=16, nx=4):
    lam0, tau, t0 = pulse_for(lams)
    prob = O.Problem(nx=nx, ny=ny, h=h, lambda0=lam0, n_steps=steps, n_pml=n_pml, dft_start=0)
    return prob, tau, t0


def tmm_rt(prob, coef, lo, hi, lam):
    """Discrete transfer matrix of rows [lo, hi) of label 1 (coef from the oracle)."""
    dt = prob.dt
    w = 2 * np.pi * C0 / lam
    z = np.exp(-1j * w * dt)
    rows = np.arange(prob.ny)
    inside = (rows >= lo) & (rows < hi)
    n_poles = (coef.shape[1] - 2) // 3
    pchi = sum(coef[1, 4 + 3 * q] / (z - coef[1, 2 + 3 * q] - coef[1, 3 + 3 * q] / z) for q in range(n_poles))
    return CF.discrete_stack_rt(np.where(inside, coef[1, 0], coef[0, 0]), np.where(inside, coef[1, 1], coef[0, 1]),
                                prob.h, dt, w, np.where(inside, pchi, 0.0))


@pytest.mark.parametrize("pole", [lorentz(2.0, 0.6, 500e-9, 0.08), [1.5, 0.0, (2 * np.pi * C0 / 300e-9) ** 2, 0.0,
                                                                     2 * np.pi * C0 / 3e-6]])
def test_discrete_susceptibility_tends_to_the_continuous_model(pole):
    """eps0 chi_d(w) = zeta / (z - alpha - xi/z), z = e^{-i w dt}, against
    eps0 a/(w_p^2 - w^2 - i g w) (Lorentz; the second case is a Drude term,
    w_p = 0); the error falls about 4x per halving of dt."""
    model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], pole])
    a, wp, g = pole[2:5]
    errs = []
    for h in (20e-9, 10e-9, 5e-9):
        prob = O.Problem(nx=4, ny=64, h=h, lambda0=600e-9, n_steps=10)
        coef = O.ade_coefficients(prob, model, 1)
        al, xi, ze = coef[1, 2:5]
        # vacuum label: no response
        assert coef[0, 4] == 0.0
        e = 0.0
        for lam in (400e-9, 550e-9, 800e-9):
            w = 2 * np.pi * C0 / lam
            z = np.exp(-1j * w * prob.dt)
            chi_d = ze / (z - al - xi / z) / O.EPS0
            chi = a / (wp * wp - w * w - 1j * g * w)
            e = max(e, abs(chi_d - chi) / abs(chi))
        errs.append(e)
    assert errs[0] < 0.05
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


@pytest.mark.parametrize("pole,n_pml,steps,tol", [
    (lorentz(2.0, 0.5, 500e-9, 0.1), 16, 5000, 5e-6),
    (lorentz(2.0, 0.5, 500e-9, 0.1), 32, 5000, 1e-6),
    (lorentz(1.8, 1.2, 620e-9, 0.02, sigma=2e4), 32, 10000, 5e-7),      # narrow pole: rings longer
    # Drude film (w_p = 0): highly reflective, so the CPML's own reflection
    # sets the residual (2e-6 with 32 cells, 2.5e-7 with 64)
    ([1.2, 0.0, (2 * np.pi * C0 / 250e-9) ** 2, 0.0, 2 * np.pi * C0 / 5e-6], 64, 10000, 5e-7),
])
def test_dispersive_slab_equals_the_discrete_steady_state(pole, n_pml, steps, tol):
    lams = np.array([450e-9, 500e-9, 550e-9, 650e-9, 800e-9, 900e-9])
    ny = 336 + 2 * n_pml
    lo, hi = ny // 2 - 50, ny // 2 + 50
    if pole[3] == 0.0:          # metal: a thin film keeps some transmission
        lo, hi = ny // 2 - 5, ny // 2 + 5
    prob, tau, t0 = slab_problem(ny, 20e-9, lams, steps, n_pml=n_pml)
    lab = np.zeros((ny, 4), np.uint8)
    lab[lo:hi] = 1
    model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], pole])
    res = O.simulate_pulse(prob, lab, model, 1, lams, tau, t0)
    for f, lam in enumerate(lams):
        R, T = tmm_rt(prob, res["coef"], lo, hi, lam)
        assert abs(res["R"][f] - R) < tol and abs(res["T"][f] - T) < tol, (lam, res["R"][f], R, res["T"][f], T)
    assert np.all(res["A"] > -tol)


def test_two_poles_add():
    """Two poles in one label: the steady state takes the sum of their responses."""
    lams = np.array([480e-9, 600e-9, 750e-9])
    prob, tau, t0 = slab_problem(360, 20e-9, lams, 10000, n_pml=32)   # the 662 nm pole rings long
    lab = np.zeros((360, 4), np.uint8)
    lab[140:220] = 1
    p1 = lorentz(1.7, 0.3, 430e-9, 0.05)
    p2 = lorentz(0.0, 0.2, 662e-9, 0.03)
    model = np.array([[1.0, 0.0] + [0.0] * 6, p1 + p2[2:]])
    res = O.simulate_pulse(prob, lab, model, 2, lams, tau, t0)
    for f, lam in enumerate(lams):
        R, T = tmm_rt(prob, res["coef"], 140, 220, lam)
        assert abs(res["R"][f] - R) < 5e-7 and abs(res["T"][f] - T) < 5e-7


def test_pulse_without_poles_equals_monochromatic_runs():
    """A label with eps_inf and a fixed sigma, no poles: the broadband run gives
    at each wavelength what the CW path gives with the same (eps_r, sigma)."""
    eps_r, sigma = 1.45 ** 2, 3e4
    lams = np.array([500e-9, 650e-9, 800e-9])
    ny, lo, hi = 300, 110, 170
    prob, tau, t0 = slab_problem(ny, 20e-9, lams, 4000, n_pml=32)
    lab = np.zeros((ny, 4), np.uint8)
    lab[lo:hi] = 1
    model = np.array([[1.0, 0.0], [eps_r, sigma]])
    res = O.simulate_pulse(prob, lab, model, 0, lams, tau, t0)
    for f, lam in enumerate(lams):
        cw = O.Problem(nx=4, ny=ny, h=20e-9, lambda0=lam, n_steps=12000, n_pml=32)
        ce_l, cb_l = O.material_eps(eps_r, sigma, cw.dt)
        ce = np.where(lab == 1, ce_l, 1.0)
        cb = np.where(lab == 1, cb_l, cw.dt / O.EPS0)
        ref = O.simulate(cw, ce=ce, cb=cb, keep_state=False)
        assert abs(res["R"][f] - ref["R"]) < 2e-5 and abs(res["T"][f] - ref["T"]) < 2e-5, (lam, res["R"][f],
                                                                                       ref["R"], res["T"][f], ref["T"])


def test_lossless_dispersive_grating_conserves_energy():
    """gamma = 0, sigma = 0: R + T = 1 at every wavelength of a random
    two-material grating (600 nm period) whose orders +-1 propagate across the
    band (455-510 nm).  The band stays clear of the Rayleigh anomaly at 600 nm,
    where a grazing order leaves the cell only as t^{-1/2} and no finite run
    converges; the poles sit in the ultraviolet, outside the pulse spectrum, as
    an undamped pole inside it would ring for ever."""
    nx, ny, h = 30, 260, 20e-9
    lab = np.zeros((ny, nx), np.uint8)
    blocks = np.random.default_rng(5).integers(1, 3, size=(12, 9))
    lab[100:120] = np.kron(blocks, np.ones((5, 5), np.uint8))[:20, :nx]
    model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(1.3, 0.3, 150e-9, 0.0), lorentz(1.6, 0.2, 150e-9, 0.0)])
    lams = np.array([455e-9, 470e-9, 490e-9, 510e-9])
    lam0, tau, t0 = pulse_for(lams)
    prob = O.Problem(nx=nx, ny=ny, h=h, lambda0=lam0, n_steps=8000, n_pml=32, dft_start=0)
    res = O.simulate_pulse(prob, lab, model, 1, lams, tau, t0)
    print("R", res["R"], "T", res["T"])
    assert np.all(np.abs(res["R"] + res["T"] - 1.0) < 5e-6)
    assert res["R"].min() > 1e-3
    assert np.abs(res["state"].ez).max() < 1e-6      # the pulse has left


def test_continuous_lorentz_slab_is_approached_at_second_order():
    pole = lorentz(2.0, 0.5, 500e-9, 0.1)
    lams = [550e-9, 700e-9]
    d = 1.0e-6
    errs = []
    for h in (20e-9, 10e-9):
        n_in = int(round(d / h))
        ny = 200 + n_in + int(round(1.2e-6 / h))
        lo = int(round(1.0e-6 / h)) + 40
        prob, tau, t0 = slab_problem(ny, h, lams, int(round(5000 * 20e-9 / h)), n_pml=32)
        lab = np.zeros((ny, 4), np.uint8)
        lab[lo:lo + n_in] = 1
        model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], pole])
        res = O.simulate_pulse(prob, lab, model, 1, np.array(lams), tau, t0)
        e = 0.0
        for f, lam in enumerate(lams):
            w = 2 * np.pi * C0 / lam
            eps = pole[0] + pole[2] / (pole[3] ** 2 - w * w - 1j * pole[4] * w)
            nn = np.sqrt(eps)
            R, T = CF.slab_rt(nn.real, nn.imag, d, lam)
            e = max(e, abs(res["R"][f] - R), abs(res["T"][f] - T))
        errs.append(e)
    assert errs[0] < 0.02 and errs[0] / errs[1] > 3.0, errs
