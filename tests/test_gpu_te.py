"""TEz (P-polarisation, eqs. 14-16) on the GPU against the FP64 oracle: slab,
random maps and narrow widths (fields within 1e-3 relative L2, R/T within
1e-4), one step from random state (layer state included), bit-identical
launch configurations, mixed TMz + TEz batches, the unpolarised average, and
the adjoint's refusal of TEz runs."""
import numpy as np
import pytest

import leafgen as LG
import oracle as O
from parity_util import problem_for, rel_l2

pytestmark = pytest.mark.gpu


def te(inst):
    inst.polarization = 1
    return inst


def oracle_te(inst, n_steps=None, dft_start=-1):
    prob = problem_for(inst, n_steps, dft_start=dft_start)
    prob.polarization = 1
    return prob, O.simulate_te(prob, inst.labels, inst.nk)


def gpu_run(fdtd, insts, n_steps, **kw):
    with fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, **kw)) as s:
        s.run()
        R, T, A = s.spectra()
        f = [s.fields(k) for k in range(len(insts))]
        m = [s.monitors(k) for k in range(len(insts))]
    return (R, T, A), f, m


def check_against_oracle(fdtd, inst, tag, **kw):
    prob, ref = oracle_te(inst)
    (R, T, A), f, m = gpu_run(fdtd, [inst], inst.n_steps, **kw)
    hz, ex, ey = f[0]
    st = ref["state"]
    errs = [rel_l2(hz, st.hz * O.ETA0), rel_l2(ex, st.ex)]
    if np.abs(st.ey).max() > 0:
        errs.append(rel_l2(ey, st.ey))
    print(tag, inst.labels.shape, kw, "rel-L2", errs, "R", R[0], ref["R"], "T", T[0], ref["T"], flush=True)
    assert max(errs) < 1e-3
    assert rel_l2(m[0], ref["mon"]) < 1e-3
    assert abs(R[0] - ref["R"]) < 1e-4 and abs(T[0] - ref["T"]) < 1e-4
    return f[0], m[0]


def test_te_slab(gpu_lib):
    inst = te(LG.configs.slab_config()[0])
    f, _ = check_against_oracle(gpu_lib, inst, "te-slab")
    assert np.abs(f[2]).max() == 0.0        # x-uniform: no Ey


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_te_random_maps(gpu_lib, seed):
    inst = te(LG.configs.random_instance(100, 170, seed, n_labels=5, steps=900, n_pml=12))
    check_against_oracle(gpu_lib, inst, "te-random", t_block=4, band_rows=24)


@pytest.mark.parametrize("nx", [1, 7, 48, 65])
def test_te_narrow_widths(gpu_lib, nx):
    inst = te(LG.configs.random_instance(nx, 60, 200 + nx, n_labels=4, steps=400, n_pml=6))
    check_against_oracle(gpu_lib, inst, "te-width", t_block=8, band_rows=16)


def test_te_launch_configurations_bit_identical(gpu_lib):
    inst = te(LG.configs.random_instance(150, 131, 5, n_labels=6, steps=203, n_pml=10))
    outs = []
    for kw in [dict(kernel=1), dict(t_block=1, band_rows=7), dict(t_block=3, band_rows=16),
               dict(t_block=8, band_rows=33), dict(t_block=5, band_rows=200), dict(t_block=8, band_rows=8),
               dict(t_block=10, band_rows=13), dict(t_block=12, band_rows=40), dict(t_block=12, band_rows=5),
               # bulk items of one workgroup (256 columns, wider than this grid)
               dict(t_block=1, band_rows=7, bulk_columns=256), dict(t_block=8, band_rows=33, bulk_columns=256),
               dict(t_block=12, band_rows=40, bulk_columns=256)]:
        _, f, m = gpu_run(gpu_lib, [inst], inst.n_steps, **kw)
        outs.append((f[0], m[0], kw))
    (a0, b0, c0), m0, _ = outs[0]
    for (a, b, c), m, kw in outs[1:]:
        assert np.array_equal(a, a0) and np.array_equal(b, b0) and np.array_equal(c, c0), kw
        assert np.array_equal(m, m0), kw


@pytest.mark.parametrize("nx", [1, 64, 231, 232, 233, 300, 465])
def test_te_workgroup_bulk_items_bit_identical(gpu_lib, nx):
    """TEz bulk items of one workgroup (the cell to the left's label and the
    edge lanes' Ey and Hz crossing between waves) against the plain sweeps,
    at widths around one and two workgroups' owned columns."""
    inst = te(LG.configs.random_instance(nx, 96, 500 + nx, n_labels=5, steps=150, n_pml=8))
    _, f0, m0 = gpu_run(gpu_lib, [inst], inst.n_steps, kernel=1)
    for kw in [dict(t_block=12, band_rows=24), dict(t_block=8, band_rows=17), dict(t_block=3, band_rows=40)]:
        _, f, m = gpu_run(gpu_lib, [inst], inst.n_steps, bulk_columns=256, **kw)
        for a, b in zip(f[0], f0[0]):
            assert np.array_equal(a, b), kw
        assert np.array_equal(m[0], m0[0]), kw


def test_mixed_polarisation_batch_equals_individual_runs(gpu_lib):
    base = [LG.configs.random_instance(nx, ny, sd, steps=240, n_pml=10)
            for nx, ny, sd in [(40, 100, 1), (130, 90, 2), (77, 150, 3)]]
    insts = [base[0], te(LG.configs.random_instance(130, 90, 2, steps=240, n_pml=10)), base[2],
             te(LG.configs.random_instance(40, 100, 1, steps=240, n_pml=10))]
    for bulk in (64, 256):
        (Rb, Tb, _), fb, _ = gpu_run(gpu_lib, insts, 240, t_block=6, band_rows=20, bulk_columns=bulk)
        for k, inst in enumerate(insts):
            (R, T, _), f, _ = gpu_run(gpu_lib, [inst], 240, t_block=6, band_rows=20)
            assert R[0] == Rb[k] and T[0] == Tb[k]
            for a, b in zip(f[0], fb[k]):
                assert np.array_equal(a, b)


@pytest.mark.parametrize("kw", [dict(kernel=1), dict(t_block=1, band_rows=9), dict(t_block=4, band_rows=16),
                                dict(t_block=12, band_rows=16), dict(t_block=4, band_rows=16, bulk_columns=256)])
def test_te_steps_from_random_state(gpu_lib, kw):
    inst = te(LG.configs.random_instance(70, 64, 11, n_labels=4, steps=40, n_pml=8))
    prob = problem_for(inst)
    prob.polarization = 1
    rng = np.random.default_rng(3)
    ny, nx = inst.labels.shape
    hz, ex, ey, pc, pe = (rng.standard_normal((ny, nx)).astype(np.float32) for _ in range(5))
    ex[0] = 0
    coefs = O.edge_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident_te(prob)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    st = O.StateTE(f64(hz) / O.ETA0, f64(ex), f64(ey), f64(pc) / prob.h, f64(pe) / (prob.h * O.ETA0))
    c_rows = np.zeros(ny, bool); c_rows[:inst.n_pml] = True; c_rows[ny - inst.n_pml:] = True
    e_rows = np.zeros(ny, bool); e_rows[1:inst.n_pml] = True; e_rows[ny - inst.n_pml + 1:] = True
    st.phz[~c_rows] = 0
    st.pex[~e_rows] = 0
    n_adv = 12
    st, _ = O.run_te(prob, coefs, e_inc, h_inc, state=st, n_begin=0, n_end=n_adv)
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=40, **kw)) as s:
        s.set_fields(0, hz, ex, ey, pc, pe)
        s.step(n_adv)
        ghz, gex, gey = s.fields(0)
    for g, o in [(ghz, st.hz * O.ETA0), (gex, st.ex), (gey, st.ey)]:
        assert np.abs(g - o).max() < 5e-5 * np.abs(o).max()


def test_unpolarised_average_against_the_oracle_of_both_polarisations(gpu_lib):
    """The library's unpolarised mean (fdtd_combine_spectra through
    fdtd.unpolarized) of a TMz and a TEz run of the same map, batched in one
    context, against the mean of the oracle's TMz and TEz runs; and a recorded
    run refuses TEz instances (the adjoint covers TMz)."""
    tm_inst = LG.configs.random_instance(64, 120, 9, steps=600, n_pml=10)
    te_inst = te(LG.configs.random_instance(64, 120, 9, steps=600, n_pml=10))
    (R, T, A), _, _ = gpu_run(gpu_lib, [tm_inst, te_inst], 600)
    Ru, Tu, Au = gpu_lib.unpolarized((R[:1], T[:1], A[:1]), (R[1:], T[1:], A[1:]))
    prob = problem_for(tm_inst)
    ref_tm = O.simulate(prob, tm_inst.labels, tm_inst.nk)
    prob_te = problem_for(te_inst)
    prob_te.polarization = 1
    ref_te = O.simulate_te(prob_te, te_inst.labels, te_inst.nk)
    Ro, To = 0.5 * (ref_tm["R"] + ref_te["R"]), 0.5 * (ref_tm["T"] + ref_te["T"])
    print("unpolarised R %.6f (oracle %.6f) T %.6f (oracle %.6f)" % (Ru[0], Ro, Tu[0], To))
    assert abs(Ru[0] - Ro) < 1e-4 and abs(Tu[0] - To) < 1e-4
    assert abs(Au[0] - (1.0 - Ro - To)) < 2e-4
    with gpu_lib.Simulation([te_inst], gpu_lib.Options(n_steps=600, checkpoint_every=-1)) as s:
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.run(record=True)
        assert e.value.code == -1
