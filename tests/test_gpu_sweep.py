"""Per-instance run lengths in one batched context, and the spectral sweep over
wavelength x polarisation x slice on the GPU: a shorter run in a batch is
bit-identical to the same run in a context of its own length (streaming and
plain kernels, graph replay, TMz and TEz), matches the FP64 oracle run for
its own length, and a multi-context sweep reproduces single runs exactly and
averages them."""
import numpy as np
import pytest

import leafgen as LG
import oracle as O
from paper_2512_17132_amd import sweep as SW
from parity_util import oracle_run, oracle_fields_normalised, problem_for, rel_l2

pytestmark = pytest.mark.gpu


def _single(fdtd, inst, n, **kw):
    with fdtd.Simulation([inst], fdtd.Options(n_steps=n, **kw)) as s:
        s.run()
        return s.spectra(), s.fields(0), s.monitors(0)


def _mixed_batch():
    insts = [LG.configs.random_instance(nx, ny, sd, n_labels=5, steps=0, n_pml=10)
             for nx, ny, sd in [(90, 120, 31), (64, 100, 32), (130, 96, 33), (50, 110, 34)]]
    insts[1].polarization = 1
    insts[3].polarization = 1
    return insts, [400, 250, 313, 400]


@pytest.mark.parametrize("kw", [dict(t_block=12, band_rows=24, use_graph=0), dict(t_block=10, band_rows=40, use_graph=1),
                                dict(t_block=5, band_rows=16, use_graph=1), dict(kernel=1)])
def test_shorter_runs_in_a_batch_equal_their_own_runs(gpu_lib, kw):
    insts, steps = _mixed_batch()
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=max(steps), **kw), run_steps=steps) as s:
        s.run()
        assert s.steps_done() == max(steps)
        R, T, A = s.spectra()
        fb = [s.fields(k) for k in range(len(insts))]
        mb = [s.monitors(k) for k in range(len(insts))]
    for k, inst in enumerate(insts):
        (r, t, _), f, m = _single(gpu_lib, inst, steps[k], **kw)
        assert R[k] == r[0] and T[k] == t[0], (k, kw)
        for a, b in zip(fb[k], f):
            assert np.array_equal(a, b), (k, kw)
        assert np.array_equal(mb[k], m), (k, kw)


def test_split_stepping_across_run_ends(gpu_lib):
    """fdtd_step calls whose boundaries straddle the instances' ends give the
    full run's result."""
    insts, steps = _mixed_batch()
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=400, t_block=8, band_rows=32), run_steps=steps) as s:
        s.run()
        ref = [s.fields(k) for k in range(len(insts))], s.spectra()
        s.reset()
        for n in (100, 151, 62, 87):
            s.step(n)
        got = [s.fields(k) for k in range(len(insts))], s.spectra()
    for a, b in zip(ref[0], got[0]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert np.array_equal(ref[1][0], got[1][0]) and np.array_equal(ref[1][1], got[1][1])


def test_shorter_run_against_the_oracle(gpu_lib):
    insts, steps = _mixed_batch()
    inst = insts[2]
    prob, ref = oracle_run(inst, n_steps=steps[2])
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=max(steps)), run_steps=steps) as s:
        s.run()
        R, T, _ = s.spectra()
        ez, hx, hy = s.fields(2)
    oez, ohx, ohy = oracle_fields_normalised(ref)
    print("short run R", R[2], ref["R"], "T", T[2], ref["T"])
    assert max(rel_l2(ez, oez), rel_l2(hx, ohx), rel_l2(hy, ohy)) < 1e-3
    assert abs(R[2] - ref["R"]) < 1e-4 and abs(T[2] - ref["T"]) < 1e-4


def test_sweep_over_slices_wavelengths_and_polarisations(gpu_lib):
    base = LG.configs.random_instance(250, 150, 41, n_labels=5, steps=0, n_pml=10, dx=25e-9)
    nk0 = base.nk.copy()

    def nk_of(lam):
        nk = nk0.copy()
        nk[1:, 1] *= 550e-9 / lam      # absorption falling with wavelength
        return nk

    lams = [450e-9, 600e-9, 900e-9]
    runs = SW.plan(base.labels, nk_of, lams, base.dx, base.n_pml, base.j_src, base.j_ref, base.j_trn,
                   SW.steps_for_periods(14, floor=300), n_slices=5)
    assert len(runs) == 30 and len({r.n_steps for r in runs}) == 3
    # the library's allocation for one run is what the planner counts
    with gpu_lib.Simulation([runs[0]], gpu_lib.Options(n_steps=runs[0].n_steps, t_block=4, band_rows=16)) as s:
        assert s.config()["device_bytes"] == SW.device_bytes(runs[0])
    per = max(SW.device_bytes(r) for r in runs)
    res = SW.run_sweep(runs, budget_bytes=8 * per)
    assert len(res.batches) >= 4
    # the first context is tuned, the later ones reuse its launch shape
    assert len(res.shapes) == len(res.batches) and len(set(res.shapes)) == 1
    assert np.all(np.abs(res.R + res.T + res.A - 1.0) < 1e-12)
    assert np.all((res.R > 0) & (res.T > 0) & (res.A > -1e-4))
    # every run equals its own single context
    for i in (0, 7, 13, 29):
        (r, t, _), _, _ = _single(gpu_lib, runs[i], runs[i].n_steps)
        assert res.R[i] == r[0] and res.T[i] == t[0], i
    lam, R, T, A = res.spectrum()
    for k, l in enumerate(lam):
        sel = [i for i, r in enumerate(runs) if r.lambda0 == l]
        assert R[k] == pytest.approx(res.R[sel].mean(), abs=1e-15)
    print("sweep spectrum", list(zip(lam, R, T, A)))
