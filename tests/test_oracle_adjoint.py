"""Oracle adjoint pins: the per-step transpose satisfies <A x, y> = <x, A^T y>
(dot-product test) and the reverse sweep matches central finite differences
of the forward oracle for per-label (n, k) and per-pixel eps_r."""
import numpy as np
import pytest

import oracle as O


def _problem(nx=24, ny=96, steps=1200):
    rng = np.random.default_rng(1)
    lab = np.zeros((ny, nx), np.uint8)
    lab[40:60] = rng.integers(1, 4, size=(20, nx))
    nk = np.array([[1.0, 0.0], [1.5, 0.02], [1.33, 0.0], [1.4, 0.05]])
    prob = O.Problem(nx=nx, ny=ny, h=20e-9, lambda0=500e-9, n_steps=steps, n_pml=12)
    return prob, lab, nk


def _random_state(prob, rng):
    pe, ph = O.cpml_profiles(prob)
    st = O.State(*(rng.standard_normal((prob.ny, prob.nx)) for _ in range(5)))
    st.hx[0] = 0.0
    st.pez[pe[:, 1] == 0] = 0.0
    st.phx[ph[:, 1] == 0] = 0.0
    st.phx[0] = 0.0
    return st


def _dot(a, b):
    return sum(float((x * y).sum()) for x, y in zip((a.ez, a.hx, a.hy, a.pez, a.phx),
                                                    (b.ez, b.hx, b.hy, b.pez, b.phx)))


def test_step_dot_product():
    prob, lab, nk = _problem()
    prob = O.Problem(**{**prob.__dict__, "dft_start": 10 ** 9})
    ce, cb = O.pixel_coefficients(prob, lab, nk)
    rng = np.random.default_rng(2)
    for _ in range(3):
        x = _random_state(prob, rng)
        y = _random_state(prob, rng)
        # scale H to SI-like magnitudes so every term contributes
        ax, _, _ = O.run(prob, ce, cb, state=x.copy(), n_begin=0, n_end=1)
        aty = O.step_adjoint(prob, ce, cb, y.copy())
        lhs, rhs = _dot(ax, y), _dot(x, aty)
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12 * abs(lhs))


@pytest.fixture(scope="module")
def grad_case():
    prob, lab, nk = _problem()
    res, gnk, geps, _ = O.gradient(prob, lab, nk, 1.0, 0.3)
    return prob, lab, nk, res, gnk, geps


def _loss(prob, lab, nk, ce=None, cb=None):
    r = O.simulate(prob, lab, nk, ce=ce, cb=cb, keep_state=False)
    return r["R"] + 0.3 * r["T"]


@pytest.mark.parametrize("label", [1, 2, 3])
@pytest.mark.parametrize("comp", [0, 1])
def test_label_gradient_vs_central_difference(grad_case, label, comp):
    prob, lab, nk, res, gnk, geps = grad_case
    h = 1e-5
    p, m = nk.copy(), nk.copy()
    p[label, comp] += h
    m[label, comp] -= h
    fd = (_loss(prob, lab, p) - _loss(prob, lab, m)) / (2 * h)
    assert gnk[label, comp] == pytest.approx(fd, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("j,i", [(45, 3), (50, 10), (30, 5), (58, 23)])
def test_pixel_eps_gradient_vs_central_difference(grad_case, j, i):
    prob, lab, nk, res, gnk, geps = grad_case
    ce, cb = res["ce"], res["cb"]
    n, k = nk[lab[j, i]]
    eps = n * n - k * k
    sig = 2 * prob.omega * O.EPS0 * n * k
    vals = []
    for s in (1, -1):
        ce2, cb2 = ce.copy(), cb.copy()
        ce2[j, i], cb2[j, i] = O.material_eps(eps + s * 1e-5, sig, prob.dt)
        vals.append(_loss(prob, lab, None, ce2, cb2))
    fd = (vals[0] - vals[1]) / 2e-5
    assert geps[j, i] == pytest.approx(fd, rel=1e-5, abs=1e-12)
