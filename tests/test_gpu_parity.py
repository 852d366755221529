"""GPU parity: the HIP library against the FP64 oracle on identical seeded
inputs (fields within 1e-3 relative L2, R/T within 1e-4 absolute), and
consistency between launch configurations (bit-identical fields)."""
import numpy as np
import pytest

import leafgen as LG
import oracle as O
from parity_util import oracle_run, problem_for, rel_l2, oracle_fields_normalised

pytestmark = pytest.mark.gpu


def _sim(fdtd, insts, n_steps, **kw):
    return fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, **kw))


def test_dpp_lane_direction_and_slab(gpu_lib):
    """Config-1 slab (256 x 256, 3000 steps): R, T against the oracle and the
    discrete transfer matrix."""
    inst = LG.configs.slab_config()[0]
    prob, ref = oracle_run(inst)
    with _sim(gpu_lib, [inst], inst.n_steps) as s:
        s.run()
        R, T, A = s.spectra()
        ez, hx, hy = s.fields(0)
    oez, ohx, ohy = oracle_fields_normalised(ref)
    print("slab R", R[0], ref["R"], "T", T[0], ref["T"])
    assert abs(R[0] - ref["R"]) < 1e-4 and abs(T[0] - ref["T"]) < 1e-4
    assert rel_l2(ez, oez) < 1e-3 and rel_l2(hx, ohx) < 1e-3
    assert np.abs(hy).max() < 1e-6 * np.abs(hx).max() + 1e-12   # x-uniform: Hy stays 0


@pytest.mark.parametrize("seed,K", [(0, 4), (1, 4), (2, 4), (3, 12)])
def test_random_map_fields_and_spectra(gpu_lib, seed, K):
    inst = LG.configs.random_instance(100, 170, seed, n_labels=5, steps=900, n_pml=12)
    prob, ref = oracle_run(inst)
    oez, ohx, ohy = oracle_fields_normalised(ref)
    with _sim(gpu_lib, [inst], inst.n_steps, t_block=K, band_rows=24) as s:
        s.run()
        R, T, A = s.spectra()
        ez, hx, hy = s.fields(0)
        mon = s.monitors(0)
    errs = [rel_l2(ez, oez), rel_l2(hx, ohx), rel_l2(hy, ohy)]
    print("seed", seed, "field rel-L2", errs, "R", R[0], ref["R"], "T", T[0], ref["T"])
    assert max(errs) < 1e-3
    assert rel_l2(mon, ref["mon"]) < 1e-3
    assert abs(R[0] - ref["R"]) < 1e-4 and abs(T[0] - ref["T"]) < 1e-4


def test_launch_configurations_bit_identical(gpu_lib):
    """Plain per-step kernels and the streaming kernel at several (K, band,
    special band) shapes give bit-identical fields and monitors (ragged nx and
    ny)."""
    inst = LG.configs.random_instance(150, 131, 5, n_labels=6, steps=203, n_pml=10)
    outs = []
    for kw in [dict(kernel=1), dict(t_block=1, band_rows=7), dict(t_block=3, band_rows=16),
               dict(t_block=8, band_rows=33), dict(t_block=5, band_rows=200), dict(t_block=8, band_rows=8),
               dict(t_block=10, band_rows=13), dict(t_block=12, band_rows=40), dict(t_block=12, band_rows=5),
               dict(t_block=10, band_rows=24, special_rows=8), dict(t_block=12, band_rows=16, special_rows=1),
               dict(t_block=7, band_rows=30, special_rows=5),
               # bulk items of one workgroup (256 columns, wider than this grid)
               dict(t_block=1, band_rows=7, bulk_columns=256), dict(t_block=8, band_rows=33, bulk_columns=256),
               dict(t_block=5, band_rows=200, bulk_columns=256), dict(t_block=12, band_rows=40, bulk_columns=256),
               dict(t_block=12, band_rows=5, bulk_columns=256),
               dict(t_block=7, band_rows=30, special_rows=5, bulk_columns=256)]:
        with _sim(gpu_lib, [inst], inst.n_steps, **kw) as s:
            s.run()
            outs.append((s.fields(0), s.monitors(0), kw))
    (e0, x0, y0), m0, _ = outs[0]
    for (e, x, y), m, kw in outs[1:]:
        assert np.array_equal(e, e0) and np.array_equal(x, x0) and np.array_equal(y, y0), kw
        assert np.array_equal(m, m0), kw


@pytest.mark.parametrize("nx", [1, 63, 64, 65, 231, 232, 233, 257, 300, 464, 465, 700])
def test_workgroup_bulk_items_bit_identical(gpu_lib, nx):
    """Bulk items of one workgroup (four waves exchanging their edge columns,
    256 - 2K columns owned) against the plain per-step kernels at widths below,
    at and past one and two workgroups' owned columns (232 and 464 at K = 12,
    240 at K = 8) and past the 256 computed columns."""
    inst = LG.configs.random_instance(nx, 96, 400 + nx, n_labels=5, steps=150, n_pml=8)
    with _sim(gpu_lib, [inst], inst.n_steps, kernel=1) as s:
        s.run()
        (e0, x0, y0), m0 = s.fields(0), s.monitors(0)
    for kw in [dict(t_block=12, band_rows=24), dict(t_block=8, band_rows=17), dict(t_block=3, band_rows=40)]:
        with _sim(gpu_lib, [inst], inst.n_steps, bulk_columns=256, **kw) as s:
            assert s.config()["bulk_columns"] == 256
            s.run()
            assert s.config()["lean_cells"] > 0
            (e, x, y), m = s.fields(0), s.monitors(0)
        assert np.array_equal(e, e0) and np.array_equal(x, x0) and np.array_equal(y, y0), kw
        assert np.array_equal(m, m0), kw


def test_split_run_equals_full_run(gpu_lib):
    inst = LG.configs.random_instance(64, 120, 7, steps=300, n_pml=10)
    with _sim(gpu_lib, [inst], inst.n_steps, t_block=4, band_rows=32) as s:
        s.run()
        full = s.fields(0)
        s.reset()
        s.step(37)
        s.step(101)
        assert s.steps_done() == 138
        s.run()
        split = s.fields(0)
    for a, b in zip(full, split):
        assert np.array_equal(a, b)


def test_batched_equals_individual(gpu_lib):
    insts = [LG.configs.random_instance(nx, ny, sd, steps=240, n_pml=10)
             for nx, ny, sd in [(40, 100, 1), (130, 90, 2), (77, 150, 3)]]
    with _sim(gpu_lib, insts, 240, t_block=6, band_rows=20) as s:
        s.run()
        Rb, Tb, _ = s.spectra()
        fb = [s.fields(k) for k in range(3)]
    for k, inst in enumerate(insts):
        with _sim(gpu_lib, [inst], 240, t_block=6, band_rows=20) as s:
            s.run()
            R, T, _ = s.spectra()
            f = s.fields(0)
        assert R[0] == Rb[k] and T[0] == Tb[k]
        for a, b in zip(f, fb[k]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("kw", [dict(kernel=1), dict(t_block=1, band_rows=9), dict(t_block=4, band_rows=16),
                                dict(t_block=12, band_rows=16), dict(t_block=1, band_rows=9, bulk_columns=256)])
def test_one_step_from_random_state(gpu_lib, kw):
    """One step from random fields (absorbing-layer state included): the raw
    update, periodic wrap and layer recursions against the oracle."""
    inst = LG.configs.random_instance(70, 64, 11, n_labels=4, steps=10, n_pml=8)
    prob = problem_for(inst)
    rng = np.random.default_rng(3)
    ny, nx = inst.labels.shape
    ez, hx, hy, pe, ph = (rng.standard_normal((ny, nx)).astype(np.float32) for _ in range(5))
    hx[0] = 0
    ce, cb = O.pixel_coefficients(prob, inst.labels, inst.nk)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    st = O.State(f64(ez), f64(hx) / O.ETA0, f64(hy) / O.ETA0, f64(pe) / (prob.h * O.ETA0), f64(ph) / prob.h)
    pe_rows = np.zeros(ny, bool); pe_rows[:inst.n_pml] = True; pe_rows[ny - inst.n_pml:] = True
    ph_rows = np.zeros(ny, bool); ph_rows[1:inst.n_pml] = True; ph_rows[ny - inst.n_pml + 1:] = True
    st.pez[~pe_rows] = 0
    st.phx[~ph_rows] = 0
    st, _, _ = O.run(prob, ce, cb, state=st, n_begin=0, n_end=1)
    with _sim(gpu_lib, [inst], 10, **kw) as s:
        s.set_fields(0, ez, hx, hy, pe, ph)
        s.step(1)
        gez, ghx, ghy = s.fields(0)
    for g, o in [(gez, st.ez), (ghx, st.hx * O.ETA0), (ghy, st.hy * O.ETA0)]:
        assert np.abs(g - o).max() < 2e-5 * np.abs(o).max()
