"""GPU edge cases: grids narrower than one 64-lane strip and ragged widths,
grids with no interior (branch-free) band at all, the full 256-entry label
table, the shortest monitor window, compensated monitor sums against an FP64
sum of the same FP32 fields, non-finite state reported as unstable, HIP
graph replays against eager launches, and sampled kernel timing."""
import numpy as np
import pytest

import leafgen as LG
from parity_util import oracle_run, rel_l2, oracle_fields_normalised

pytestmark = pytest.mark.gpu


def _sim(fdtd, insts, n_steps, **kw):
    return fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, **kw))


def _compare_to_oracle(fdtd, inst, tag, **kw):
    prob, ref = oracle_run(inst)
    oez, ohx, ohy = oracle_fields_normalised(ref)
    with _sim(fdtd, [inst], inst.n_steps, **kw) as s:
        s.run()
        R, T, A = s.spectra()
        ez, hx, hy = s.fields(0)
        mon = s.monitors(0)
    errs = [rel_l2(ez, oez), rel_l2(hx, ohx)] + ([rel_l2(hy, ohy)] if np.abs(ohy).max() > 0 else [])
    print(tag, inst.labels.shape, kw, "rel-L2", errs, "R", R[0], ref["R"], "T", T[0], ref["T"], flush=True)
    assert max(errs) < 1e-3
    assert rel_l2(mon, ref["mon"]) < 1e-3
    assert abs(R[0] - ref["R"]) < 1e-4 and abs(T[0] - ref["T"]) < 1e-4
    return ez, hx, hy, mon


@pytest.mark.parametrize("nx,K", [(1, 8), (2, 8), (7, 8), (47, 8), (48, 8), (49, 8), (63, 8), (64, 8), (65, 8),
                                  (129, 8), (1, 12), (39, 12), (40, 12), (41, 12), (81, 12)])
def test_narrow_and_ragged_widths(gpu_lib, nx, K):
    """Widths below, at and just past one strip (64 - 2K written columns: 48
    at K = 8, 40 at K = 12), wrapping inside a single wave; plain and
    streaming kernels bit-identical."""
    inst = LG.configs.random_instance(nx, 60, 100 + nx, n_labels=4, steps=400, n_pml=6)
    a = _compare_to_oracle(gpu_lib, inst, "width", t_block=K, band_rows=16)
    with _sim(gpu_lib, [inst], inst.n_steps, kernel=1) as s:
        s.run()
        b = s.fields(0) + (s.monitors(0),)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_grid_without_interior_band(gpu_lib):
    """ny = 28 with 4-cell layers: every row is within K rows of a layer, the
    TF/SF line or a monitor, so only the special-band variant runs."""
    inst = LG.configs.random_instance(80, 28, 3, n_labels=3, steps=300, n_pml=4)
    for K in (8, 12):
        with _sim(gpu_lib, [inst], inst.n_steps, t_block=K, band_rows=64) as s:
            assert s.config()["lean_cells"] == 0
        _compare_to_oracle(gpu_lib, inst, "no-interior", t_block=K, band_rows=64)


def test_full_label_table(gpu_lib):
    inst = LG.configs.random_instance(96, 140, 21, n_labels=256, steps=600, n_pml=10, block=(2, 2))
    assert inst.labels.max() > 200
    _compare_to_oracle(gpu_lib, inst, "256-labels", t_block=6, band_rows=32)


def test_shortest_monitor_window(gpu_lib):
    inst = LG.configs.random_instance(64, 100, 8, steps=500, n_pml=8)
    import oracle as O
    from parity_util import problem_for
    prob = problem_for(inst, dft_start=inst.n_steps - 2)
    ref = O.simulate(prob, inst.labels, inst.nk)
    with _sim(gpu_lib, [inst], inst.n_steps, dft_start=inst.n_steps - 2) as s:
        s.run()
        R, T, _ = s.spectra()
        mon = s.monitors(0)
    assert rel_l2(mon, ref["mon"]) < 1e-4
    assert R[0] == pytest.approx(ref["R"], rel=1e-3, abs=1e-4)
    assert T[0] == pytest.approx(ref["T"], rel=1e-3, abs=1e-4)


def test_compensated_monitor_sums_match_fp64_sum_of_the_same_fields(gpu_lib):
    """The monitor accumulators (eqs. 29-30) against an FP64 sum, on the host,
    of the very FP32 fields the GPU produced on the two monitor rows, step by
    step, times the FP32 phasors cos/sin(w (n + 1/2) dt)."""
    inst = LG.configs.random_instance(64, 100, 4, steps=4000, n_pml=8)
    n0 = 1000
    s1 = inst.courant / np.sqrt(2.0)
    wdt = 2.0 * np.pi * s1 * inst.dx / inst.lambda0
    ref = np.zeros((4, inst.nx))
    with _sim(gpu_lib, [inst], inst.n_steps, dft_start=n0) as s:
        s.step(n0)
        for n in range(n0, inst.n_steps):
            s.step(1)
            ez = s.fields(0)[0].astype(np.float64)
            c = np.float64(np.float32(np.cos(wdt * (n + 0.5))))
            sn = np.float64(np.float32(np.sin(wdt * (n + 0.5))))
            ref[0] += ez[inst.j_ref] * c
            ref[1] += ez[inst.j_ref] * sn
            ref[2] += ez[inst.j_trn] * c
            ref[3] += ez[inst.j_trn] * sn
        mon = s.monitors(0)
    for r in range(4):
        err = np.abs(mon[r] - ref[r]).max() / np.abs(ref[r]).max()
        print("monitor", r, "max relative error", err)
        assert err < 1e-6


def test_nonfinite_state_is_reported_as_unstable(gpu_lib):
    inst = LG.configs.random_instance(64, 100, 6, steps=40, n_pml=8)
    with _sim(gpu_lib, [inst], inst.n_steps, dft_start=1) as s:
        ez = np.zeros(inst.labels.shape, np.float32)
        ez[inst.j_ref, 5] = np.nan
        s.set_fields(0, ez=ez)
        s.run()
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.spectra()
        assert e.value.code == -6
        # a reset clears the state and the flag
        s.reset()
        s.run()
        R, T, A = s.spectra()
        assert np.isfinite(R).all() and np.isfinite(T).all()


@pytest.mark.parametrize("bulk", [64, 256])
def test_graph_replays_match_eager_launches(gpu_lib, bulk):
    """A captured full run replayed several times, with eager device work and
    a partial eager run of the same context between replays, gives exactly the
    fields, monitors and spectra of an eager run every time (bulk bands as
    items of one wave and of one workgroup)."""
    import torch
    insts = [LG.configs.random_instance(nx, ny, sd, steps=333, n_pml=10)
             for nx, ny, sd in [(90, 130, 31), (300, 96, 32)]]
    with _sim(gpu_lib, insts, 333, t_block=8, band_rows=32, use_graph=0, bulk_columns=bulk) as s:
        s.run()
        want = ([s.fields(k) for k in range(2)], [s.monitors(k) for k in range(2)], s.spectra())
    with _sim(gpu_lib, insts, 333, t_block=8, band_rows=32, use_graph=1, bulk_columns=bulk) as s:
        for rep in range(4):
            if rep:
                s.reset()
            s.run()
            got = ([s.fields(k) for k in range(2)], [s.monitors(k) for k in range(2)], s.spectra())
            for k in range(2):
                for a, b in zip(got[0][k], want[0][k]):
                    assert np.array_equal(a, b), rep
                assert np.array_equal(got[1][k], want[1][k]), rep
            for a, b in zip(got[2], want[2]):
                assert np.array_equal(a, b), rep
            # eager work between replays: torch kernels on the same stream and a
            # partial run of this context that does not use the graph
            x = torch.randn(1 << 20, device="cuda")
            torch.cuda.synchronize()
            assert torch.isfinite(x.sum()).item()
            s.reset()
            s.step(17)
            s.run()
            for k in range(2):
                assert np.array_equal(s.fields(k)[0], want[0][k][0])


@pytest.mark.parametrize("every", [1, 3, 8])
def test_sampled_kernel_timing_counts_and_leaves_results_unchanged(gpu_lib, every):
    """Timing every N-th bulk launch: ceil(launches / N) launches timed, a
    positive duration, and fields bit-identical to an untimed run."""
    inst = LG.configs.random_instance(150, 200, 41, steps=8 * 25, n_pml=12)
    with _sim(gpu_lib, [inst], inst.n_steps, t_block=8, band_rows=32, use_graph=0) as s:
        s.run()
        want = s.fields(0)
    with _sim(gpu_lib, [inst], inst.n_steps, t_block=8, band_rows=32, use_graph=0) as s:
        s.set_profiling(True, every=every)
        s.run()
        ms, n = s.kernel_time()
        s.set_profiling(False)
        got = s.fields(0)
    assert n == -(-25 // every) and ms > 0
    for a, b in zip(got, want):
        assert np.array_equal(a, b)


def test_autotune_table_keeps_constrained_choices_apart(gpu_lib):
    """The autotuner's process-wide table of chosen launch shapes: a shape
    chosen with t_block fixed is not handed to a context that leaves it free
    (that context runs its own trials), and a second free context reuses the
    free choice without trials (best rate 0)."""
    inst = LG.configs.random_instance(77, 133, 61, n_labels=3, steps=120, n_pml=10)

    def tune(**kw):
        with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=120, use_graph=0, **kw)) as s:
            rate = s.autotune()
            cfg = s.config()
            return rate, (cfg["t_block"], cfg["band_rows"], cfg["special_rows"], cfg["bulk_columns"])

    r_fixed, c_fixed = tune(t_block=2)
    assert r_fixed > 0 and c_fixed[0] == 2
    r_free, c_free = tune()
    assert r_free > 0
    r_again, c_again = tune()
    assert r_again == 0 and c_again == c_free
