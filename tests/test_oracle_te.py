"""Pins of the TEz (P-polarisation) oracle, eqs. 14-16: the discrete transfer
matrix of the Ex recurrence with edge-averaged materials, second-order
convergence to the continuous slab (at normal incidence TE and TM share the
Fresnel result), energy balance of a lossless grating with the TEz order
weights w_m = tan(ky_0 h/2)/tan(ky_m h/2), TF/SF leakage, the empty domain,
and periodic-shift and mirror symmetry."""
import numpy as np
import pytest

import oracle as O
from closed_forms import discrete_stack_rt, slab_rt


def _slab(ny=256, nx=4, lo=103, hi=153):
    lab = np.zeros((ny, nx), np.uint8)
    lab[lo:hi] = 1
    return lab


def _te(**kw):
    kw.setdefault("polarization", 1)
    return O.Problem(**kw)


def test_slab_matches_discrete_transfer_matrix_with_edge_averaged_materials():
    nk = np.array([[1.0, 0.0], [1.45, 0.01]])
    prob = _te(nx=4, ny=256, h=20e-9, lambda0=600e-9, n_steps=3000, n_pml=16)
    r = O.simulate_te(prob, _slab(), nk)
    cex, cbx, _, _ = r["coefs"]
    Rd, Td = discrete_stack_rt(cex[1:, 0], cbx[1:, 0], prob.h, prob.dt, prob.omega)
    assert abs(r["R"] - Rd) < 1e-5 and abs(r["T"] - Td) < 1e-5
    # the interface edges carry the mean of vacuum and slab
    assert 1.0 > cex[103, 0] > cex[104, 0] and cbx[103, 0] > cbx[104, 0]


def test_thick_layers_reach_the_discrete_steady_state_closer():
    nk = np.array([[1.0, 0.0], [1.6, 0.03]])
    prob = _te(nx=4, ny=320, h=20e-9, lambda0=550e-9, n_steps=6000, n_pml=32)
    r = O.simulate_te(prob, _slab(320, 4, 130, 190), nk)
    cex, cbx, _, _ = r["coefs"]
    Rd, Td = discrete_stack_rt(cex[1:, 0], cbx[1:, 0], prob.h, prob.dt, prob.omega)
    assert abs(r["R"] - Rd) < 1e-6 and abs(r["T"] - Td) < 1e-6


def test_second_order_convergence_to_the_continuous_slab():
    Rc, Tc = slab_rt(1.45, 0.01, 1.0e-6, 600e-9)
    errs = []
    for h in (20e-9, 10e-9):
        d = int(round(1.0e-6 / h))
        ny = int(round(5.12e-6 / h))
        lo = ny // 2 - d // 2
        prob = _te(nx=2, ny=ny, h=h, lambda0=600e-9, n_steps=int(3000 * 20e-9 / h), n_pml=int(16 * 20e-9 / h))
        r = O.simulate_te(prob, _slab(ny, 2, lo, lo + d), np.array([[1.0, 0.0], [1.45, 0.01]]))
        errs.append(abs(r["R"] - Rc) + abs(r["T"] - Tc))
    assert errs[1] < errs[0] / 3.0


def _grating(nx=112, ny=256, seed=0):
    rng = np.random.default_rng(seed)
    lab = np.zeros((ny, nx), np.uint8)
    blk = rng.integers(0, 3, size=(10, -(-nx // 8)))
    lab[90:170] = np.kron(blk, np.ones((8, 8), np.uint8))[:80, :nx]
    return lab


@pytest.fixture(scope="module")
def lossless_grating_te():
    nk = np.array([[1.0, 0.0], [1.5, 0.0], [1.3, 0.0]])
    prob = _te(nx=112, ny=256, h=20e-9, lambda0=600e-9, n_steps=16000, n_pml=32)
    return prob, O.simulate_te(prob, _grating(), nk)


def test_lossless_grating_conserves_energy_with_te_weights(lossless_grating_te):
    prob, r = lossless_grating_te
    w = r["orders"]["w"]
    assert (w > 0).sum() >= 5
    assert w.min(where=w > 0, initial=10) == pytest.approx(1.0)     # m = 0 has the smallest TEz weight
    assert abs(r["R"] + r["T"] - 1.0) < 2e-5


def test_unit_weights_break_te_energy_balance(lossless_grating_te):
    prob, r = lossless_grating_te
    p2 = O.Problem(**{**prob.__dict__, "literal_orders": 1})
    R, T, A, _ = O.spectra(p2, r["mon"], r["inc"])
    assert abs(R + T - 1.0) > 0.02


def test_te_tfsf_line_does_not_leak():
    ny, nx = 256, 8
    prob = _te(nx=nx, ny=ny, h=20e-9, lambda0=600e-9, n_steps=3000, n_pml=16)
    coefs = O.edge_coefficients(prob, np.zeros((ny, nx), np.uint8), np.array([[1.0, 0.0]]))
    e_inc, h_inc = O.incident_te(prob)
    n_a = 2 * prob.aux_pad - 8
    st, _ = O.run_te(prob, coefs, e_inc, h_inc, n_end=n_a)
    sf = np.abs(st.ex[prob.j_src + 1:]).max()
    tf = np.abs(st.ex[: prob.j_src + 1]).max()
    assert tf > 0.05 and sf < 1e-13 * tf
    assert np.abs(st.ey).max() == 0.0          # x-uniform: no Ey


def test_te_empty_domain_transmits_and_layers_absorb():
    prob = _te(nx=4, ny=256, h=20e-9, lambda0=600e-9, n_steps=3000, n_pml=16)
    r = O.simulate_te(prob, np.zeros((256, 4), np.uint8), np.array([[1.0, 0.0]]))
    assert np.sqrt(r["R"]) < 1e-4
    assert abs(r["T"] - 1.0) < 2e-5


def test_te_periodic_shift_and_mirror_symmetry():
    nk = np.array([[1.0, 0.0], [1.5, 0.03], [1.3, 0.01]])
    lab = _grating(nx=64, seed=5)
    prob = _te(nx=64, ny=256, h=20e-9, lambda0=600e-9, n_steps=2500, n_pml=16)
    a = O.simulate_te(prob, lab, nk)
    b = O.simulate_te(prob, np.roll(lab, 17, axis=1), nk)
    assert b["R"] == pytest.approx(a["R"], rel=1e-11, abs=1e-14)
    assert b["T"] == pytest.approx(a["T"], rel=1e-11, abs=1e-14)
    half = _grating(nx=32, seed=7)
    sym = np.concatenate([half, half[:, ::-1]], axis=1)
    r = O.simulate_te(_te(nx=64, ny=256, h=20e-9, lambda0=450e-9, n_steps=2500, n_pml=16), sym, nk)
    m, ref = r["orders"]["m"], r["orders"]["ref"]
    for mm in range(1, 4):
        assert ref[m == mm][0] == pytest.approx(ref[m == -mm][0], rel=1e-9, abs=1e-15)
