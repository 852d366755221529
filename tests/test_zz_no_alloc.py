"""fdtd_step_noalloc (stepping with the work-item lists in the library's fixed
device array, no device allocation) against fdtd_step: fields and monitor
sums bit-identical, on two calls in a row, the second on a smaller input; and
its refusals (no settled launch shape, a launch above the array's size)."""
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
