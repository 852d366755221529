"""Host logic of the spectral sweep (slices, run plan, run-length rule, packing
under a memory budget, averaging); no GPU needed."""
import math

import numpy as np
import pytest

from paper_2512_17132_amd import sweep as SW


@pytest.mark.parametrize("nx,n", [(10, 1), (10, 3), (8511, 5), (7, 7), (1703, 5)])
def test_slices_tile_the_width(nx, n):
    b = SW.slice_bounds(nx, n)
    assert len(b) == n and b[0][0] == 0 and b[-1][1] == nx
    assert all(b[k][1] == b[k + 1][0] for k in range(n - 1))
    widths = [x1 - x0 for x0, x1 in b]
    assert max(widths) - min(widths) <= 1 and min(widths) >= 1


def test_slice_count_above_width_is_rejected():
    with pytest.raises(ValueError):
        SW.slice_bounds(4, 5)


def test_steps_per_period_matches_the_time_step():
    # dt = S dx / (c sqrt 2): at S = 1, dx = 0.01 m the paper's validation step
    # is 23.57 ps; one period of lambda = 1 m is then lambda / (c dt) steps
    dx, S, lam, c = 0.01, 1.0, 1.0, 299792458.0
    dt = S * dx / (c * math.sqrt(2.0))
    assert SW.steps_per_period(lam, dx, S) == pytest.approx(lam / c / dt, rel=1e-12)
    rule = SW.steps_for_periods(10, floor=100)
    n = rule(lam, dx, S)
    assert n % 2 == 0 and n >= 10 * SW.steps_per_period(lam, dx, S)
    assert rule(1e-3, dx, S) == 100


def _labels(ny=60, nx=50):
    lab = np.zeros((ny, nx), np.uint8)
    lab[20:40, ::3] = 1
    return lab


def test_plan_covers_every_slice_wavelength_and_polarisation():
    lab = _labels()
    lams = [500e-9, 600e-9, 700e-9]
    runs = SW.plan(lab, lambda lam: np.array([[1.0, 0.0], [1.5, lam * 1e4]]), lams, 20e-9, 8, 52, 56, 12,
                   SW.steps_for_periods(20), n_slices=5)
    assert len(runs) == 5 * 3 * 2
    keys = {(r.slice, r.lambda0, r.polarization) for r in runs}
    assert len(keys) == 30
    for r in runs:
        x0, x1 = SW.slice_bounds(50, 5)[r.slice]
        assert np.array_equal(r.labels, lab[:, x0:x1]) and r.labels.flags.c_contiguous
        assert r.nk[1, 1] == pytest.approx(r.lambda0 * 1e4)
    # runs of one slice share one label array
    assert runs[0].labels is runs[5].labels
    # longer wavelengths get longer runs under a periods rule
    by_lam = {r.lambda0: r.n_steps for r in runs}
    assert by_lam[500e-9] < by_lam[600e-9] < by_lam[700e-9]


def test_device_bytes_counts_fields_layers_labels_and_tables():
    r = SW.Run(np.zeros((100, 70), np.uint8), np.ones((1, 2)), 20e-9, 500e-9, 8, 80, 90, 12, 0, 1000)
    pitch = 128
    fields = 2 * 3 * 100 * pitch * 4
    layers = 2 * 2 * 17 * pitch * 4
    assert fields + layers + 100 * pitch < SW.device_bytes(r) < fields + layers + 100 * pitch + 40000


def test_pack_respects_the_budget_and_groups_similar_lengths():
    lab = _labels()
    runs = SW.plan(lab, lambda lam: np.array([[1.0, 0.0], [1.5, 0.0]]), [400e-9, 800e-9, 1600e-9], 20e-9, 8,
                   52, 56, 12, SW.steps_for_periods(10), n_slices=2)
    per = max(SW.device_bytes(r) for r in runs)
    batches = SW.pack(runs, 5 * per)
    assert sorted(i for b in batches for i in b) == list(range(len(runs)))
    for b in batches:
        assert sum(SW.device_bytes(runs[i]) for i in b) <= 5 * per
    # longest runs first
    firsts = [runs[b[0]].n_steps for b in batches]
    assert firsts == sorted(firsts, reverse=True)
    with pytest.raises(ValueError):
        SW.pack(runs, per // 2)


def test_spectrum_averages_slices_and_polarisations():
    lab = _labels()
    runs = SW.plan(lab, lambda lam: np.array([[1.0, 0.0], [1.5, 0.0]]), [500e-9, 700e-9], 20e-9, 8, 52, 56, 12,
                   400, n_slices=3)
    rng = np.random.default_rng(0)
    R, T = rng.uniform(0, 0.5, len(runs)), rng.uniform(0, 0.5, len(runs))
    res = SW.SweepResult(runs, R, T, 1 - R - T, [list(range(len(runs)))])
    lams, Rm, Tm, Am = res.spectrum()
    for k, lam in enumerate(lams):
        sel = [i for i, r in enumerate(runs) if r.lambda0 == lam]
        assert len(sel) == 6
        assert Rm[k] == pytest.approx(R[sel].mean()) and Tm[k] == pytest.approx(T[sel].mean())
        assert Am[k] == pytest.approx(1 - R[sel].mean() - T[sel].mean())
    _, Rs, _, _ = res.spectrum(polarizations=[0])
    sel = [i for i, r in enumerate(runs) if r.lambda0 == lams[0] and r.polarization == 0]
    assert Rs[0] == pytest.approx(R[sel].mean())
