"""Oracle pins for x-invariant stacks: the exact steady state of the discrete
recurrence (open vacuum and finite column with absorbing layers) and O(h^2)
convergence to the continuous slab (Fresnel + Fabry-Perot)."""
import numpy as np
import pytest

import closed_forms as CF
import oracle as O


def _slab(ny, nx, lo, hi, n, k, dx, lam, steps, n_pml):
    prob = O.Problem(nx=nx, ny=ny, h=dx, lambda0=lam, n_steps=steps, n_pml=n_pml)
    lab = np.zeros((ny, nx), np.uint8)
    lab[lo:hi] = 1
    return prob, O.simulate(prob, lab, np.array([[1.0, 0.0], [n, k]]))


@pytest.fixture(scope="module")
def config1():
    # 256 x 256 at 20 nm, 1.0 um slab n = 1.45 + 0.01i, lambda = 600 nm, 3000 steps
    return _slab(256, 256, 103, 153, 1.45, 0.01, 20e-9, 600e-9, 3000, 16)


def test_config1_discrete_transfer_matrix(config1):
    prob, r = config1
    R, T = CF.discrete_stack_rt(r["ce"][:, 0], r["cb"][:, 0], prob.h, prob.dt, prob.omega)
    assert R == pytest.approx(0.026050, abs=1e-6) and T == pytest.approx(0.780143, abs=1e-6)
    # 16 CPML cells leave a reflection amplitude of ~6e-6, which bounds the agreement
    assert abs(r["R"] - R) < 1e-5 and abs(r["T"] - T) < 1e-5
    assert r["A"] == pytest.approx(1 - R - T, abs=2e-5)


def test_thick_cpml_discrete_transfer_matrix():
    prob, r = _slab(288, 2, 119, 169, 1.45, 0.01, 20e-9, 600e-9, 3000, 32)
    R, T = CF.discrete_stack_rt(r["ce"][:, 0], r["cb"][:, 0], prob.h, prob.dt, prob.omega)
    assert abs(r["R"] - R) < 1e-6 and abs(r["T"] - T) < 1e-6


def test_config1_full_column_steady_state(config1):
    """Frequency-domain solve of the same finite column, absorbing layers and
    TF/SF line included: the time-domain run must reach it to ~1e-8."""
    prob, r = config1
    pe, ph = O.cpml_profiles(prob)
    E = CF.column_steady_state(r["ce"][:, 0], r["cb"][:, 0], pe, ph, prob.h, prob.dt, prob.omega, prob.j_src)
    assert abs(r["R"] - abs(E[prob.j_ref]) ** 2) < 5e-8
    assert abs(r["T"] - abs(E[prob.j_trn]) ** 2) < 5e-8
    # the steady-state field itself, column by column
    e_row = r["state"].ez[:, 0]
    assert np.isfinite(e_row).all()


@pytest.mark.parametrize("n,k,lam", [(1.5, 0.0, 550e-9), (1.36, 0.05, 450e-9), (1.7, 0.3, 700e-9)])
def test_full_column_other_stacks(n, k, lam):
    prob, r = _slab(240, 2, 100, 137, n, k, 20e-9, lam, 4000, 16)
    pe, ph = O.cpml_profiles(prob)
    E = CF.column_steady_state(r["ce"][:, 0], r["cb"][:, 0], pe, ph, prob.h, prob.dt, prob.omega, prob.j_src)
    assert abs(r["R"] - abs(E[prob.j_ref]) ** 2) < 5e-8
    assert abs(r["T"] - abs(E[prob.j_trn]) ** 2) < 5e-8


def test_second_order_convergence_to_continuous_slab():
    Rc, Tc = CF.slab_rt(1.45, 0.01, 1.0e-6, 600e-9)
    assert Rc == pytest.approx(0.029413, abs=1e-6) and Tc == pytest.approx(0.779326, abs=1e-6)
    errs = []
    for dx, ny, steps in [(20e-9, 256, 3000), (10e-9, 512, 6000)]:
        cells = int(round(1.0e-6 / dx))
        lo = ny // 2 - cells // 2
        prob, r = _slab(ny, 2, lo, lo + cells, 1.45, 0.01, dx, 600e-9, steps, 16 * int(20e-9 / dx))
        errs.append(np.hypot(r["R"] - Rc, r["T"] - Tc))
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, (errs, ratio)
