"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the autotuner picks for them (the one the benchmark times).

A full run of those grids is out of the oracle's reach in a test, so each case
fills every cell with random fields (absorbing-layer state included), advances
two streaming launches' worth of steps with the source and the monitors live,
and compares with the oracle advanced from the same state: fields within
1e-5 relative L2 (FP32 against FP64 over 2K steps) and the monitor sums
likewise.  The batched workload is checked on sampled instances (the largest
and smallest grids of each geometry) inside the full 122-instance launch, and
the 8192 x 16384 workload (4 wavelengths x 2 geometries in one launch) on one
instance of each geometry.  The broadband form of the batched workload (two
full-size leaves with two-pole dispersive labels and 61 monitor wavelengths in
one context) runs from zero fields until the pulse is inside the leaf, against
the oracle's dispersive path over the same steps; so does the healthy leaf in
broadband TEz."""
import os

import numpy as np
import pytest

import leafgen as LG
import oracle as O
from parity_util import problem_for, rel_l2

pytestmark = pytest.mark.gpu


def random_state(inst, rng):
    ny, nx = inst.labels.shape
    ez, hx, hy, pe, ph = (rng.standard_normal((ny, nx), dtype=np.float32) for _ in range(5))
    hx[0] = 0
    return ez, hx, hy, pe, ph


def oracle_from_state(inst, state, n_steps_total, dft_start, n_adv):
    """The oracle advanced n_adv steps from a normalised-unit state."""
    prob = problem_for(inst, n_steps_total, dft_start=dft_start)
    ez, hx, hy, pe, ph = state
    ny, nx = inst.labels.shape
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    st = O.State(f64(ez), f64(hx) / O.ETA0, f64(hy) / O.ETA0, f64(pe) / (prob.h * O.ETA0), f64(ph) / prob.h)
    pe_rows = np.zeros(ny, bool)
    pe_rows[:inst.n_pml] = True
    pe_rows[ny - inst.n_pml:] = True
    ph_rows = np.zeros(ny, bool)
    ph_rows[1:inst.n_pml] = True
    ph_rows[ny - inst.n_pml + 1:] = True
    st.pez[~pe_rows] = 0
    st.phx[~ph_rows] = 0
    ce, cb = O.pixel_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident(prob)
    st, mon, _ = O.run(prob, ce, cb, e_inc, h_inc, state=st, n_begin=0, n_end=n_adv)
    return st, mon


def check(sim, k, inst, state, n_steps, dft_start, n_adv, tag):
    st, mon = oracle_from_state(inst, state, n_steps, dft_start, n_adv)
    ez, hx, hy = sim.fields(k)
    errs = [rel_l2(ez, st.ez), rel_l2(hx, st.hx * O.ETA0), rel_l2(hy, st.hy * O.ETA0)]
    merr = rel_l2(sim.monitors(k), mon)
    print(tag, inst.name, inst.labels.shape, "field rel-L2", errs, "monitor rel-L2", merr, flush=True)
    assert max(errs) < 1e-5, errs
    assert merr < 1e-5, merr


def test_dicot_full_size_from_random_state(gpu_lib):
    inst = LG.configs.dicot_config()[0]
    assert inst.labels.shape == (8192, 4096)
    dft_start = 1
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps, dft_start=dft_start)) as s:
        s.autotune()
        cfg = s.config()
        print("dicot launch configuration", cfg, flush=True)
        assert cfg["kernel"] == 0 and cfg["t_block"] >= 1
        state = random_state(inst, np.random.default_rng(2024))
        s.set_fields(0, *state)
        n_adv = 2 * cfg["t_block"]
        s.step(n_adv)
        check(s, 0, inst, state, inst.n_steps, dft_start, n_adv, "dicot")


def test_batched_full_launch_sampled_instances(gpu_lib):
    steps = 20000
    insts = LG.configs.batched_config_parallel(steps, workers=min(16, os.cpu_count() or 1))
    assert len(insts) == 122
    sizes = [i.cells for i in insts]
    sample = sorted({0, 60, 61, 121, int(np.argmax(sizes)), int(np.argmin(sizes))})
    dft_start = 1
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=steps, dft_start=dft_start)) as s:
        s.autotune()
        cfg = s.config()
        print("batched launch configuration", cfg, flush=True)
        rng = np.random.default_rng(77)
        states = {}
        for k in sample:
            states[k] = random_state(insts[k], rng)
            s.set_fields(k, *states[k])
        n_adv = 2 * cfg["t_block"]
        s.step(n_adv)
        for k in sample:
            check(s, k, insts[k], states[k], steps, dft_start, n_adv, "batched")


def test_large_full_launch_sampled_instances(gpu_lib):
    """The 8 instances of 8192 x 16384 cells (1.07e9 cells) in one context, at
    the autotuned launch shape; a random state on the first instance of each
    geometry (450 nm healthy, 850 nm diseased), against the oracle."""
    insts = LG.configs.large_config_parallel()
    assert len(insts) == 8 and all(i.labels.shape == (16384, 8192) for i in insts)
    sample = [0, 7]
    dft_start = 1
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=insts[0].n_steps, dft_start=dft_start)) as s:
        s.autotune()
        cfg = s.config()
        print("large launch configuration", cfg, flush=True)
        rng = np.random.default_rng(8192)
        states = {}
        for k in sample:
            states[k] = random_state(insts[k], rng)
            s.set_fields(k, *states[k])
        n_adv = 2 * cfg["t_block"]
        s.step(n_adv)
        for k in sample:
            check(s, k, insts[k], states[k], insts[0].n_steps, dft_start, n_adv, "large")
            del states[k]


def test_dicot_full_size_te_from_random_state(gpu_lib):
    """The TEz streaming kernel at the dicot's full size (random Hz, Ex, Ey and
    layer state, two launches) against the TEz oracle."""
    inst = LG.configs.dicot_config()[0]
    inst.polarization = 1
    dft_start = 1
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps, dft_start=dft_start)) as s:
        s.autotune()
        cfg = s.config()
        print("dicot TEz launch configuration", cfg, flush=True)
        rng = np.random.default_rng(4048)
        ny, nx = inst.labels.shape
        hz, ex, ey, pc, pe = (rng.standard_normal((ny, nx), dtype=np.float32) for _ in range(5))
        ex[0] = 0
        s.set_fields(0, hz, ex, ey, pc, pe)
        n_adv = 2 * cfg["t_block"]
        s.step(n_adv)
        ghz, gex, gey = s.fields(0)
        gmon = s.monitors(0)
    prob = problem_for(inst, inst.n_steps, dft_start=dft_start)
    prob.polarization = 1
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    st = O.StateTE(f64(hz) / O.ETA0, f64(ex), f64(ey), f64(pc) / prob.h, f64(pe) / (prob.h * O.ETA0))
    c_rows = np.zeros(ny, bool); c_rows[:inst.n_pml] = True; c_rows[ny - inst.n_pml:] = True
    e_rows = np.zeros(ny, bool); e_rows[1:inst.n_pml] = True; e_rows[ny - inst.n_pml + 1:] = True
    st.phz[~c_rows] = 0
    st.pex[~e_rows] = 0
    coefs = O.edge_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident_te(prob)
    st, mon = O.run_te(prob, coefs, e_inc, h_inc, state=st, n_begin=0, n_end=n_adv)
    errs = [rel_l2(ghz, st.hz * O.ETA0), rel_l2(gex, st.ex), rel_l2(gey, st.ey)]
    merr = rel_l2(gmon, mon)
    print("dicot TEz field rel-L2", errs, "monitor rel-L2", merr, flush=True)
    assert max(errs) < 1e-5 and merr < 1e-5


def test_broadband_full_size_against_the_oracle(gpu_lib):
    """Both broadband leaves (1831 x 3662 and 2048 x 4096 cells, 2 poles, 61
    wavelengths) in one context at the autotuned launch shape, 2400 steps from
    zero fields.  By then the pulse reflected by the leaf surface has crossed
    the reflection line (its peak arrives after about 1800 steps), while the
    transmission line, about 4000 rows below the source, is still outside the
    scheme's light cone.  Fields, and the reflection line's sums at every
    wavelength, within 1e-3 relative L2 of the oracle; the transmission line's
    sums exactly zero on both sides."""
    n = 2400
    insts = [LG.configs.broadband_leaf(steps=20000, geometry=g) for g in ("healthy", "diseased")]
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=20000)) as s:
        s.autotune()
        cfg = s.config()
        print("broadband launch configuration", cfg, flush=True)
        s.step(n)
        got = [(s.fields(k), s.monitors(k)) for k in range(2)]
    for inst, (fields, mon) in zip(insts, got):
        ny, nx = inst.labels.shape
        assert ny - inst.n_pml - 8 - (inst.n_pml + 4) > n       # the transmission line is out of reach
        prob = O.Problem(nx=nx, ny=ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps, n_pml=inst.n_pml,
                         j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn, courant=inst.courant, dft_start=0)
        coef = O.ade_coefficients(prob, inst.model, inst.n_poles)
        e_inc, h_inc = O.incident_pulse(prob, inst.pulse_tau, inst.pulse_t0)
        st, omon = O.run_ade(prob, inst.labels, coef, inst.n_poles, inst.lambdas, e_inc, h_inc, n_end=n)
        errs = [rel_l2(fields[0], st.ez), rel_l2(fields[1], st.hx * O.ETA0), rel_l2(fields[2], st.hy * O.ETA0)]
        merr = [rel_l2(mon[f, :2], omon[f, :2]) for f in range(len(inst.lambdas))]
        print("broadband", inst.name, (ny, nx), "field rel-L2", errs, "reflection-line rel-L2 worst / median",
              max(merr), float(np.median(merr)), "max |Ez|", float(np.abs(st.ez).max()), flush=True)
        assert np.abs(st.ez).max() > 1e-3
        assert max(errs) < 1e-3 and max(merr) < 1e-3
        assert not omon[:, 2:].any() and not mon[:, 2:].any()


def test_broadband_te_full_size_against_the_oracle(gpu_lib):
    """The healthy broadband leaf (1831 x 3662 cells, 2 poles, 61 wavelengths)
    in TEz, on the streaming kernel at the autotuned launch shape, 2400 steps
    from zero fields: fields and the reflection line's sums at every
    wavelength within 1e-3 relative L2 of the oracle's dispersive TEz path;
    the transmission line's sums exactly zero on both sides."""
    n = 2400
    inst = LG.configs.broadband_leaf(steps=20000, geometry="healthy")
    inst.polarization = 1
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=20000)) as s:
        s.autotune()
        cfg = s.config()
        assert cfg["kernel"] == 0
        print("broadband TEz launch shape", cfg["t_block"], cfg["band_rows"], cfg["special_rows"], flush=True)
        s.step(n)
        fields, mon = s.fields(0), s.monitors(0)
    ny, nx = inst.labels.shape
    prob = O.Problem(nx=nx, ny=ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps, n_pml=inst.n_pml,
                     j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn, courant=inst.courant, dft_start=0,
                     polarization=1)
    coef = O.ade_coefficients(prob, inst.model, inst.n_poles)
    edge = O.edge_model_coefficients(prob, inst.labels, inst.model, inst.n_poles)
    e_inc, h_inc = O.incident_pulse(prob, inst.pulse_tau, inst.pulse_t0)
    st, omon = O.run_te_ade(prob, inst.labels, coef, edge, inst.n_poles, inst.lambdas, e_inc, h_inc, n_end=n)
    errs = [rel_l2(fields[0], st.hz * O.ETA0), rel_l2(fields[1], st.ex), rel_l2(fields[2], st.ey)]
    merr = [rel_l2(mon[f, :2], omon[f, :2]) for f in range(len(inst.lambdas))]
    print("broadband TEz", (ny, nx), "field rel-L2", errs, "reflection-line rel-L2 worst / median", max(merr),
          float(np.median(merr)), "max |Ex|", float(np.abs(st.ex).max()), flush=True)
    assert np.abs(st.ex).max() > 1e-3
    assert max(errs) < 1e-3 and max(merr) < 1e-3
    assert not omon[:, 2:].any() and not mon[:, 2:].any()
