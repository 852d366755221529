"""Pins of the oracle's dispersive TEz path (broadband P polarisation, the
TEz update of eqs. 14-16 with the Lorentz-Drude labels of Sec. 2.2).  Reading:
an edge's permittivity is the mean of its two cells' at every frequency, so
its (Ce, Cb) come from the mean eps_inf and sigma and its polarisation is half
the sum of both cells' pole responses to the edge field.

* a pulsed TEz run of a dispersive slab equals, at every monitor wavelength,
  the exact steady state of the discrete scheme: the transfer matrix of the Ex
  recurrence with edge coefficients and the edge-averaged discrete
  susceptibility;
* with no poles, the pulsed TEz run equals monochromatic TEz runs of the
  pinned CW path at each wavelength;
* a lossless dispersive grating conserves energy under the TEz order weights;
* refined grids approach the continuous Lorentz slab at second order (at
  normal incidence TE and TM share the Fresnel result)."""
import numpy as np

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


def te_problem(ny, h, lams, steps, n_pml=32, nx=4):
    lam0, tau, t0 = pulse_for(lams)
    prob = O.Problem(nx=nx, ny=ny, h=h, lambda0=lam0, n_steps=steps, n_pml=n_pml, dft_start=0, polarization=1)
    return prob, tau, t0


def discrete_chi(coef_row, n_poles, z):
    """P/E of one label's pole recursions at z = exp(-i w dt)."""
    return sum(coef_row[4 + 3 * q] / (z - coef_row[2 + 3 * q] - coef_row[3 + 3 * q] / z) for q in range(n_poles))


def slab_tmm(prob, res, lab_col, n_poles, lam):
    """Discrete transfer matrix of the Ex recurrence of one column: edge rows
    1.. with their (Ce, Cb) and the mean of the two cells' susceptibilities."""
    w = 2 * np.pi * C0 / lam
    z = np.exp(-1j * w * prob.dt)
    chi = np.array([discrete_chi(res["coef"][L], n_poles, z) for L in range(res["coef"].shape[0])])
    cex, cbx, _, _ = res["edge"]
    pchi = 0.5 * (chi[lab_col[1:]] + chi[lab_col[:-1]])
    return CF.discrete_stack_rt(cex[1:, 0], cbx[1:, 0], prob.h, prob.dt, w, pchi)


def test_dispersive_te_slab_equals_the_discrete_steady_state():
    lams = np.array([450e-9, 500e-9, 550e-9, 650e-9, 800e-9, 900e-9])
    for pole, tol in ((lorentz(2.0, 0.5, 500e-9, 0.1), 1e-6),
                      (lorentz(1.8, 1.2, 620e-9, 0.02, sigma=2e4), 5e-7)):
        ny = 400
        prob, tau, t0 = te_problem(ny, 20e-9, lams, 10000)
        lab = np.zeros((ny, 4), np.uint8)
        lab[150:250] = 1
        model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], pole])
        res = O.simulate_pulse(prob, lab, model, 1, lams, tau, t0)
        for f, lam in enumerate(lams):
            R, T = slab_tmm(prob, res, lab[:, 0], 1, lam)
            assert abs(res["R"][f] - R) < tol and abs(res["T"][f] - T) < tol, (lam, res["R"][f], R, res["T"][f], T)
        # the interface edge (between cells 149 and 150) takes the mean eps_inf
        _, cbx, _, _ = res["edge"]
        assert cbx[149, 0] > cbx[150, 0] > cbx[151, 0]
        assert np.isclose(1 / cbx[150, 0], 0.5 * (1 / cbx[149, 0] + 1 / cbx[151, 0]), rtol=1e-3)


def test_two_poles_in_a_te_slab():
    lams = np.array([480e-9, 600e-9, 750e-9])
    prob, tau, t0 = te_problem(360, 20e-9, lams, 10000)
    lab = np.zeros((360, 4), np.uint8)
    lab[140:220] = 1
    p1 = lorentz(1.7, 0.3, 430e-9, 0.05)
    p2 = lorentz(0.0, 0.2, 662e-9, 0.03)
    model = np.array([[1.0, 0.0] + [0.0] * 6, p1 + p2[2:]])
    res = O.simulate_pulse(prob, lab, model, 2, lams, tau, t0)
    for f, lam in enumerate(lams):
        R, T = slab_tmm(prob, res, lab[:, 0], 2, lam)
        assert abs(res["R"][f] - R) < 5e-7 and abs(res["T"][f] - T) < 5e-7


def test_pole_free_te_pulse_equals_monochromatic_te_runs():
    """eps_inf and a fixed sigma with no poles: each wavelength of the pulsed
    TEz run equals a CW TEz run with the same (eps_r, sigma), i.e. with
    (n, k) from n^2 - k^2 = eps_r and 2 n k = sigma/(w eps0)."""
    eps_r, sigma = 1.45 ** 2, 3e4
    lams = np.array([500e-9, 650e-9, 800e-9])
    ny, lo, hi = 300, 110, 170
    prob, tau, t0 = te_problem(ny, 20e-9, lams, 4000)
    lab = np.zeros((ny, 4), np.uint8)
    lab[lo:hi] = 1
    res = O.simulate_pulse(prob, lab, np.array([[1.0, 0.0], [eps_r, sigma]]), 0, lams, tau, t0)
    for f, lam in enumerate(lams):
        w = 2 * np.pi * C0 / lam
        e2 = sigma / (w * O.EPS0)
        n = np.sqrt(0.5 * (eps_r + np.hypot(eps_r, e2)))
        cw = O.Problem(nx=4, ny=ny, h=20e-9, lambda0=lam, n_steps=12000, n_pml=32, polarization=1)
        ref = O.simulate_te(cw, lab, np.array([[1.0, 0.0], [n, e2 / (2 * n)]]))
        assert abs(res["R"][f] - ref["R"]) < 2e-5 and abs(res["T"][f] - ref["T"]) < 2e-5, (lam, res["R"][f],
                                                                                       ref["R"], res["T"][f], ref["T"])


def test_lossless_dispersive_te_grating_conserves_energy():
    """gamma = 0, sigma = 0, UV poles: R + T = 1 at every wavelength of a
    random two-material grating with orders +-1 propagating (TEz weights)."""
    nx, ny, h = 30, 260, 20e-9
    lab = np.zeros((ny, nx), np.uint8)
    blocks = np.random.default_rng(5).integers(1, 3, size=(12, 9))
    lab[100:120] = np.kron(blocks, np.ones((5, 5), np.uint8))[:20, :nx]
    model = np.array([[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(1.3, 0.3, 150e-9, 0.0), lorentz(1.6, 0.2, 150e-9, 0.0)])
    lams = np.array([455e-9, 470e-9, 490e-9, 510e-9])
    lam0, tau, t0 = pulse_for(lams)
    prob = O.Problem(nx=nx, ny=ny, h=h, lambda0=lam0, n_steps=8000, n_pml=32, dft_start=0, polarization=1)
    res = O.simulate_pulse(prob, lab, model, 1, lams, tau, t0)
    print("R", res["R"], "T", res["T"])
    assert np.all(np.abs(res["R"] + res["T"] - 1.0) < 5e-6)
    assert res["R"].min() > 1e-3
    assert np.abs(res["state"].ex).max() < 1e-6


def test_te_continuous_lorentz_slab_is_approached_at_second_order():
    pole = lorentz(2.0, 0.5, 500e-9, 0.1)
    lams = [550e-9, 700e-9]
    d = 1.0e-6
    errs = []
    for h in (20e-9, 10e-9):
        n_in = int(round(d / h))
        ny = 200 + n_in + int(round(1.2e-6 / h))
        lo = int(round(1.0e-6 / h)) + 40
        prob, tau, t0 = te_problem(ny, h, lams, int(round(5000 * 20e-9 / h)))
        lab = np.zeros((ny, 4), np.uint8)
        lab[lo:lo + n_in] = 1
        res = O.simulate_pulse(prob, lab, np.array([[1.0, 0.0, 0.0, 0.0, 0.0], pole]), 1, np.array(lams), tau, t0)
        e = 0.0
        for f, lam in enumerate(lams):
            w = 2 * np.pi * C0 / lam
            nn = np.sqrt(pole[0] + pole[2] / (pole[3] ** 2 - w * w - 1j * pole[4] * w))
            R, T = CF.slab_rt(nn.real, nn.imag, d, lam)
            e = max(e, abs(res["R"][f] - R), abs(res["T"][f] - T))
        errs.append(e)
    assert errs[0] < 0.02 and errs[0] / errs[1] > 3.0, errs
