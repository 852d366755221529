"""fdtd_step_noalloc (stepping with the work-item lists in the library's fixed
device array, no device allocation) against fdtd_step: fields and monitor
sums bit-identical, on two calls in a row, the second on a smaller input, and
on broadband instances of both polarisations; and its refusals (no settled
launch shape, a launch above the array's size)."""
import numpy as np
import pytest

import leafgen as LG

pytestmark = pytest.mark.gpu


def _state(sim, n_inst):
    return [(sim.fields(k), sim.monitors(k)) for k in range(n_inst)]


def _same(a, b):
    for (fa, ma), (fb, mb) in zip(a, b):
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)
        assert np.array_equal(ma, mb)


def _compare(fdtd, insts, steps, chunks, run_steps=None, **kw):
    """Steps one context with fdtd_step and another with fdtd_step_noalloc in
    the same chunks; both must agree bit for bit, fields and monitors."""
    opts = fdtd.Options(n_steps=steps, use_graph=0, **kw)
    with fdtd.Simulation(insts, opts, run_steps=run_steps) as ref:
        for n in chunks:
            ref.step(n)
        a = _state(ref, len(insts))
        spec_a = ref.spectra()
    with fdtd.Simulation(insts, opts, run_steps=run_steps) as s:
        for n in chunks:
            s.step_noalloc(n)
        assert s.steps_done() == sum(chunks)
        b = _state(s, len(insts))
        spec_b = s.spectra()
    _same(a, b)
    assert np.array_equal(spec_a[0], spec_b[0]) and np.array_equal(spec_a[1], spec_b[1])
    return a


def test_noalloc_stepping_matches_fdtd_step(gpu_lib):
    # first call: a mixed batch (TMz and TEz, ragged sizes, uneven run lengths
    # so that launches switch between lists and tail launches use other K)
    insts = [LG.configs.random_instance(nx, ny, sd, n_labels=5, steps=0, n_pml=10)
             for nx, ny, sd in [(150, 131, 51), (64, 100, 52), (97, 120, 53)]]
    insts[1].polarization = 1
    steps = [330, 250, 301]
    st = _compare(gpu_lib, insts, 330, [101, 150, 79], run_steps=steps, t_block=8, band_rows=24)
    assert all(np.abs(f[0]).max() > 0 for f, _ in st)
    # second call, right after: a smaller input, another launch shape
    small = [LG.configs.random_instance(40, 70, 54, n_labels=3, steps=0, n_pml=8)]
    _compare(gpu_lib, small, 120, [57, 63], t_block=6, band_rows=16)
    # bulk bands as workgroup items, wider than one workgroup, both polarisations
    wide = [LG.configs.random_instance(300, 90, 56, n_labels=4, steps=0, n_pml=8),
            LG.configs.random_instance(300, 90, 57, n_labels=4, steps=0, n_pml=8)]
    wide[1].polarization = 1
    _compare(gpu_lib, wide, 100, [40, 60], t_block=8, band_rows=20, bulk_columns=256)


def test_noalloc_after_autotune_and_plain_kernel(gpu_lib):
    inst = LG.configs.random_instance(130, 110, 55, steps=200, n_pml=10)
    # the launch shape settled by the autotuner
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=200, use_graph=0)) as ref:
        ref.autotune()
        ref.step(200)
        a = _state(ref, 1)
        cfg = ref.config()
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=200, use_graph=0, t_block=cfg["t_block"],
                                                    band_rows=cfg["band_rows"])) as s:
        s.step_noalloc(200)
        _same(a, _state(s, 1))
    # the plain sweeps take no list
    _compare(gpu_lib, [inst], 200, [200], kernel=1)


def _pole(d_eps, lam_p, gamma_rel):
    wp = 2 * np.pi * 299792458.0 / lam_p
    return [d_eps * wp * wp, wp, gamma_rel * wp]


def test_noalloc_broadband_both_polarisations(gpu_lib):
    """Broadband TMz and TEz instances in one context, two poles, monitors at
    three wavelengths: the TEz instance's special and lean items share one
    kernel launch and the monitor sums follow it.  Stepping through the fixed
    array matches fdtd_step bit for bit, fields and monitor sums."""
    from types import SimpleNamespace
    model = np.array([[1.0, 0.0] + [0.0] * 6,
                      [1.8, 1e4] + _pole(0.3, 480e-9, 0.1) + _pole(0.1, 700e-9, 0.05),
                      [2.1, 0.0] + _pole(0.5, 560e-9, 0.08) + _pole(0.0, 650e-9, 0.1)])
    lams = np.array([450e-9, 550e-9, 700e-9])
    lam0, tau, t0 = gpu_lib.pulse_for_band(lams.min(), lams.max())
    insts = []
    for pol, (nx, ny, sd) in enumerate([(150, 120, 58), (97, 130, 59)]):
        lab = LG.configs.random_instance(nx, ny, sd, n_labels=3, steps=0, n_pml=10).labels
        insts.append(SimpleNamespace(labels=lab, model=model, n_poles=2, lambdas=lams, pulse_tau=tau, pulse_t0=t0,
                                     lambda0=lam0, dx=20e-9, courant=0.99, n_pml=10, j_src=ny - 18,
                                     j_ref=ny - 14, j_trn=14, n_steps=500, polarization=pol))
    # the pulse peaks near step 400; spectra per wavelength from the broadband
    # monitor sums (the single-wavelength spectra do not apply)
    opts = gpu_lib.Options(n_steps=500, use_graph=0, t_block=5, band_rows=24, special_rows=8)
    out = []
    for noalloc in (False, True):
        with gpu_lib.Simulation(insts, opts) as s:
            for n in (230, 270):
                s.step_noalloc(n) if noalloc else s.step(n)
            out.append((_state(s, 2), [s.broadband_spectra(k) for k in range(2)]))
    (a, spec_a), (b, spec_b) = out
    _same(a, b)
    assert all(np.abs(m).max() > 0 for _, m in a)
    for x, y in zip(spec_a, spec_b):
        assert np.isfinite(x[0]).all() and np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_noalloc_refusals(gpu_lib):
    inst = LG.configs.random_instance(64, 90, 56, steps=100, n_pml=10)
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=100, use_graph=0)) as s:
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.step_noalloc(10)                 # no launch shape yet
        assert e.value.code == -5
        assert s.steps_done() == 0
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.step_noalloc(101)
        assert e.value.code == -1
    # 8192 columns in strips of 64 - 2*12 = 40 and 4096 rows in bands of 16:
    # 205 x 256 items, above the array's 32768
    big = LG.configs.random_instance(8192, 4096, 57, steps=24, n_pml=10)
    with gpu_lib.Simulation([big], gpu_lib.Options(n_steps=24, use_graph=0, t_block=12, band_rows=16)) as s:
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.step_noalloc(12)
        assert e.value.code == -1 and "32768" in str(e.value)
        assert s.steps_done() == 0
        s.step(12)                             # the allocating path still takes it
        assert s.steps_done() == 12
