"""The seeded leaf workloads run from zero fields to their last step on the
GPU, in the launch shape the autotuner picks (the one the benchmark times),
against the FP64 oracle run over the same steps on the same inputs:
reflectance and transmittance within 1e-4 (eqs. 31-34 with the tone fit and
flux weights), final fields and monitor sums within 1e-3 relative L2.

  - the monocot of the differentiation form, 1024 x 2048 cells, 8000 steps,
    in TMz and in TEz;
  - the three smallest instances of the batched form inside the full
    122-instance launch (61 wavelengths x 2 geometries, 20000 steps);
  - the dicot of the plain form, 4096 x 8192 cells, 20000 steps (the oracle
    takes a few minutes on the host's threads; the test reports its progress).
"""
import os
import time

import numpy as np
import pytest

import leafgen as LG
import oracle as O
from parity_util import oracle_fields_normalised, problem_for, rel_l2

pytestmark = pytest.mark.gpu

RT_TOL = 1e-4
FIELD_TOL = 1e-3


def oracle_full_run(inst, say=None, chunk=2000):
    """The oracle's run of inst from zero fields (steps in chunks, so that a
    long run can report its progress)."""
    prob = problem_for(inst)
    ce, cb = O.pixel_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident(prob)
    state, mon = None, None
    t0 = time.perf_counter()
    for n0 in range(0, prob.n_steps, chunk):
        n1 = min(prob.n_steps, n0 + chunk)
        state, mon, _ = O.run(prob, ce, cb, e_inc, h_inc, state=state, n_begin=n0, n_end=n1, mon=mon)
        if say:
            say("  oracle %s: step %d of %d (%.0f s)" % (inst.name, n1, prob.n_steps, time.perf_counter() - t0))
    inc = O.incident_sums(prob, e_inc)
    R, T, A, _ = O.spectra(prob, mon, inc)
    return dict(R=R, T=T, A=A, mon=mon, state=state)


def compare(tag, inst, R, T, fields, mon, ref):
    oez, ohx, ohy = oracle_fields_normalised(ref)
    ferr = [rel_l2(fields[0], oez), rel_l2(fields[1], ohx), rel_l2(fields[2], ohy)]
    merr = rel_l2(mon, ref["mon"])
    dR, dT = abs(R - ref["R"]), abs(T - ref["T"])
    print("%s %s %s: R %.6f (oracle %.6f, |dR| %.2e)  T %.6f (oracle %.6f, |dT| %.2e)  field rel-L2 %s  "
          "monitor rel-L2 %.2e" % (tag, inst.name, inst.labels.shape, R, ref["R"], dR, T, ref["T"], dT,
                                   ["%.2e" % e for e in ferr], merr), flush=True)
    assert dR < RT_TOL and dT < RT_TOL, (dR, dT)
    assert max(ferr) < FIELD_TOL, ferr
    assert merr < FIELD_TOL, merr
    assert R >= 0 and T >= 0 and R + T <= 1 + 1e-6


def test_monocot_full_run_against_the_oracle(gpu_lib, progress):
    inst = LG.configs.monocot_config()[0]
    assert inst.labels.shape == (2048, 1024) and inst.n_steps == 8000
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps)) as s:
        s.autotune()
        print("monocot launch configuration", s.config(), flush=True)
        s.run()
        R, T, _ = s.spectra()
        fields, mon = s.fields(0), s.monitors(0)
    progress("monocot: GPU run done, oracle running")
    ref = oracle_full_run(inst, progress)
    compare("monocot", inst, R[0], T[0], fields, mon, ref)


def test_batched_smallest_instances_full_run_against_the_oracle(gpu_lib, progress):
    steps = 20000
    insts = LG.configs.batched_config_parallel(steps, workers=min(16, os.cpu_count() or 1))
    assert len(insts) == 122
    order = np.argsort([i.cells for i in insts], kind="stable")
    sample = [int(k) for k in order[:3]]
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=steps)) as s:
        s.autotune()
        print("batched launch configuration", s.config(), flush=True)
        s.run()
        R, T, _ = s.spectra()
        got = {k: (s.fields(k), s.monitors(k)) for k in sample}
    progress("batched: GPU run of 122 instances done, oracle on %s" % [insts[k].name for k in sample])
    for k in sample:
        ref = oracle_full_run(insts[k], progress, chunk=5000)
        compare("batched", insts[k], R[k], T[k], got[k][0], got[k][1], ref)


@pytest.mark.slow
def test_dicot_full_run_against_the_oracle(gpu_lib, progress):
    inst = LG.configs.dicot_config()[0]
    assert inst.labels.shape == (8192, 4096) and inst.n_steps == 20000
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps)) as s:
        s.autotune()
        print("dicot launch configuration", s.config(), flush=True)
        s.run()
        R, T, _ = s.spectra()
        fields, mon = s.fields(0), s.monitors(0)
    progress("dicot: GPU run done (R %.6f T %.6f); oracle running on %d threads" % (R[0], T[0], O.num_threads()))
    ref = oracle_full_run(inst, progress)
    compare("dicot", inst, R[0], T[0], fields, mon, ref)


def test_monocot_te_full_run_against_the_oracle(gpu_lib, progress):
    """The monocot in TEz (P polarisation: Hz, Ex, Ey, edge-averaged
    materials) from zero fields to its last step, against the oracle's TEz
    path."""
    import copy
    inst = copy.copy(LG.configs.monocot_config()[0])
    inst.polarization = 1
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps)) as s:
        s.autotune()
        print("monocot TEz launch configuration", s.config(), flush=True)
        s.run()
        R, T, _ = s.spectra()
        (ghz, gex, gey), gmon = s.fields(0), s.monitors(0)
    progress("monocot TEz: GPU run done, oracle running")
    prob = problem_for(inst)
    prob.polarization = 1
    coefs = O.edge_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident_te(prob)
    st, mon = None, None
    for n0 in range(0, prob.n_steps, 2000):
        st, mon = O.run_te(prob, coefs, e_inc, h_inc, state=st, n_begin=n0, n_end=min(prob.n_steps, n0 + 2000), mon=mon)
    Ro, To, _, _ = O.spectra(prob, mon, O.incident_sums(prob, e_inc))
    ferr = [rel_l2(ghz, st.hz * O.ETA0), rel_l2(gex, st.ex), rel_l2(gey, st.ey)]
    merr = rel_l2(gmon, mon)
    print("monocot TEz: R %.6f (oracle %.6f)  T %.6f (oracle %.6f)  field rel-L2 %s  monitor rel-L2 %.2e"
          % (R[0], Ro, T[0], To, ["%.2e" % e for e in ferr], merr), flush=True)
    assert abs(R[0] - Ro) < RT_TOL and abs(T[0] - To) < RT_TOL
    assert max(ferr) < FIELD_TOL and merr < FIELD_TOL
    assert R[0] >= 0 and T[0] >= 0 and R[0] + T[0] <= 1 + 1e-6
