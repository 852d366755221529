"""bench.py's counter post-processing on synthetic rocprofv3 counter files:
FETCH_SIZE / WRITE_SIZE of the bulk kernel scaled by the reference copy's
reading, the TMz and TEz records kept apart, and a record ignored once the
kernel source hash differs (host logic only, no GPU)."""
import csv
import json
import os

import pytest

import bench

COPY_KIB = bench.COPY_BYTES / 1024.0


def write_pass(d, counter, kib_bulk, kib_special, copy_kib, pol, K=10, B=192, lean_cells=1000, workload=None,
               bulk_columns=None):
    os.makedirs(os.path.join(d, "run"), exist_ok=True)
    rows = []
    tm = "void fdtd::k_tblock<%d, %s, false>(fdtd::InstDev const*, int)"
    te = "void fdtd::k_tblock_te<%d, %s>(fdtd::InstDev const*, int)"
    bb = "void fdtd::k_tblock_bb<%d, %s>(fdtd::InstDev const*, int)"
    wg = "void fdtd::k_tblock_wg<%d, %s>(fdtd::InstDev const*, int)"
    name = bb if workload else te if pol else wg if bulk_columns == 256 else tm
    t = 0
    for v in kib_bulk:
        rows.append((name % (K, "false"), v, t, t + 100))
        t += 200
    for v in kib_special:   # special items: excluded
        rows.append((name % (K, "true"), v, t, t + 50))
        t += 200
    # the other polarisation's bulk kernel, and the other bulk layout's: excluded
    rows.append(((tm if pol else te) % (K, "false"), 1e9, t, t + 100))
    t += 200
    rows.append(((tm if bulk_columns == 256 else wg) % (K, "false"), 1e9, t, t + 100))
    t += 200
    rows.append(("__amd_rocclr_copyBuffer", 3.0, t, t + 10))       # a short copy (not the reference)
    t += 200
    rows.append(("__amd_rocclr_copyBuffer", copy_kib, t, t + 5000))  # the reference copy: the longest
    with open(os.path.join(d, "run", "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"])
        for k, v, a, b in rows:
            w.writerow([k, counter, v, a, b])
    with open(d + ".log", "w") as f:
        f.write("[bench] noise\n")
        info = {"profile_pass": True, "workload": workload or "dicot4096x8192", "polarization": pol,
                "t_block": K, "band_rows": B, "lean_cells": lean_cells, "launches": len(kib_bulk),
                "copy_bytes": bench.COPY_BYTES}
        if workload:
            info["bytes_per_cell"] = 57
        if bulk_columns:
            info["bulk_columns"] = bulk_columns
        f.write(json.dumps(info) + "\n")


@pytest.fixture
def sandbox(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda workload="": "h1")
    return tmp_path


def test_derive_traffic_scales_by_the_reference_copy(sandbox):
    f, w = str(sandbox / "fetch"), str(sandbox / "write")
    # FETCH_SIZE reads the 1 GiB copy as half of it, WRITE_SIZE as all of it
    write_pass(f, "FETCH_SIZE", [100.0, 300.0], [7.0], COPY_KIB / 2, pol=0)
    write_pass(w, "WRITE_SIZE", [50.0, 50.0], [9.0], COPY_KIB, pol=0)
    bench.derive_traffic(f, w)
    rec = json.load(open(sandbox / "profiles" / "traffic.json"))["dicot4096x8192"]["K10_B192"]
    c = rec["counters"]
    assert c["FETCH_SIZE"]["dispatches"] == 2 and c["WRITE_SIZE"]["dispatches"] == 2
    assert c["FETCH_SIZE"]["scale"] == pytest.approx(2.0) and c["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    assert c["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(200.0 * 2.0 * 1024)
    assert c["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx((400.0 + 50.0) * 1024)
    assert rec["algorithmic_bytes_per_launch"] == bench.BYTES_PER_CELL_LAUNCH * 1000
    assert rec["kernel_hash"] == "h1"
    assert bench.traffic_record("dicot4096x8192", 10, 192) == pytest.approx(450.0 * 1024)
    assert bench.traffic_record("dicot4096x8192", 12, 128) is None          # no record of that shape
    assert bench.traffic_record("dicot4096x8192_te", 10, 192) is None


def test_te_record_is_kept_apart_and_stale_hashes_are_ignored(sandbox, monkeypatch):
    f, w = str(sandbox / "fetch"), str(sandbox / "write")
    write_pass(f, "FETCH_SIZE", [10.0], [], COPY_KIB / 2, pol=0)
    write_pass(w, "WRITE_SIZE", [10.0], [], COPY_KIB, pol=0)
    bench.derive_traffic(f, w)
    ft, wt = str(sandbox / "fetch_te"), str(sandbox / "write_te")
    write_pass(ft, "FETCH_SIZE", [20.0, 40.0], [1.0], COPY_KIB / 2, pol=1)
    write_pass(wt, "WRITE_SIZE", [30.0, 30.0], [1.0], COPY_KIB, pol=1)
    bench.derive_traffic(ft, wt)
    allrec = json.load(open(sandbox / "profiles" / "traffic.json"))
    assert set(allrec) == {"dicot4096x8192", "dicot4096x8192_te"}
    assert bench.traffic_record("dicot4096x8192", 10, 192) == pytest.approx(30.0 * 1024)
    assert bench.traffic_record("dicot4096x8192_te", 10, 192) == pytest.approx((60.0 + 30.0) * 1024)
    # after a kernel change the recorded counters no longer describe the kernel
    monkeypatch.setattr(bench, "kernel_source_hash", lambda workload="": "h2")
    assert bench.traffic_record("dicot4096x8192", 10, 192) is None
    assert bench.traffic_record("dicot4096x8192_te", 10, 192) is None


def test_broadband_record_counts_its_own_kernel_and_bytes(sandbox):
    f, w = str(sandbox / "fetch_bb"), str(sandbox / "write_bb")
    write_pass(f, "FETCH_SIZE", [80.0, 120.0], [3.0], COPY_KIB / 2, pol=0, K=10, B=128, workload="broadband_leaves")
    write_pass(w, "WRITE_SIZE", [60.0, 60.0], [3.0], COPY_KIB, pol=0, K=10, B=128, workload="broadband_leaves")
    bench.derive_traffic(f, w)
    rec = json.load(open(sandbox / "profiles" / "traffic.json"))["broadband_leaves"]["K10_B128"]
    assert rec["algorithmic_bytes_per_launch"] == 57 * 1000
    assert rec["bytes_per_launch"] == pytest.approx((200.0 + 60.0) * 1024)
    assert bench.traffic_record("broadband_leaves", 10, 128) == pytest.approx(260.0 * 1024)
    assert bench.traffic_record("dicot4096x8192", 10, 128) is None


def test_workgroup_bulk_kernel_record_is_kept_apart(sandbox):
    """Counters of the bulk kernel whose items are workgroups count that
    kernel only and are recorded under their own shape key."""
    f, w = str(sandbox / "fetch_wg"), str(sandbox / "write_wg")
    write_pass(f, "FETCH_SIZE", [40.0, 60.0], [2.0], COPY_KIB / 2, pol=0, K=12, B=512, bulk_columns=256)
    write_pass(w, "WRITE_SIZE", [70.0, 70.0], [2.0], COPY_KIB, pol=0, K=12, B=512, bulk_columns=256)
    bench.derive_traffic(f, w)
    rec = json.load(open(sandbox / "profiles" / "traffic.json"))["dicot4096x8192"]["K12_B512_W256"]
    assert rec["bulk_columns"] == 256
    assert rec["bytes_per_launch"] == pytest.approx((100.0 + 70.0) * 1024)
    assert bench.traffic_record("dicot4096x8192", 12, 512, 256) == pytest.approx(170.0 * 1024)
    assert bench.traffic_record("dicot4096x8192", 12, 512) is None           # the one-wave layout's: absent
    assert bench.bulk_kernel_name(12, 256) == "k_tblock_wg<12,false>"
    assert bench.bulk_kernel_name(10) == "k_tblock<10,false,false>"


def test_missing_bulk_dispatches_raise(sandbox):
    f, w = str(sandbox / "fetch"), str(sandbox / "write")
    write_pass(f, "FETCH_SIZE", [], [5.0], COPY_KIB / 2, pol=0)
    write_pass(w, "WRITE_SIZE", [], [5.0], COPY_KIB, pol=0)
    with pytest.raises(RuntimeError):
        bench.derive_traffic(f, w)


def test_broadband_launch_bytes_count_driven_poles_only():
    """Algorithmic bytes of a broadband launch: 25 B per owned cell plus 16 B
    per driven pole; TEz counts both edges' first sides and, where the labels
    differ, the second cell's (below for Ex, to the left for Ey, wrapping in
    x).  Values worked out by hand on a 2 x 2 map."""
    import types
    import numpy as np
    model = np.zeros((3, 8))
    model[:, 0] = 1.0
    model[1, 2] = 1.0                        # label 1: pole 0 only
    model[2, 2], model[2, 5] = 1.0, 2.0      # label 2: both poles; label 0: none
    lab = np.array([[0, 1], [2, 2]], np.uint8)
    tm = types.SimpleNamespace(labels=lab, model=model, n_poles=2)
    # driven poles per cell 0, 1, 2, 2
    assert bench.broadband_launch_bytes([tm], 4) == 25 * 4 + 16 * 5
    te = types.SimpleNamespace(labels=lab, model=model, n_poles=2, polarization=1)
    # (0,0): 0 + left label 1 (1 pole); (0,1): 2 x 1, left label 0 (none);
    # (1,0): 2 x 2, below label 0 (none), left same label; (1,1): 2 x 2, below label 1 (1)
    assert bench.broadband_launch_bytes([te], 4) == 25 * 4 + 16 * (1 + 2 + 4 + 5)
    # two instances add; fewer owned cells lower only the field share
    assert bench.broadband_launch_bytes([tm, te], 3) == 25 * 3 + 16 * (5 + 12)
    # the broadband TEz kernel's launch also holds the special items: every
    # cell, and the two CPML states of each cell in the absorbing layers
    te.nx, te.ny, te.n_pml = 2, 2, 1
    assert bench.broadband_te_launch_bytes(te) == 25 * 4 + 16 * (1 + 2 + 4 + 5) + 16 * 2 * 1 * 2


def test_broadband_te_record_counts_every_dispatch_of_its_one_kernel(sandbox):
    """Broadband TEz runs its special and lean items in one kernel,
    k_tblock_bt<K> (no SPECIAL argument): the record averages that kernel's
    dispatches and prices them at the cells of both kinds (kernel_cells)."""
    for counter, vals, copy_kib in (("FETCH_SIZE", [30.0, 50.0], COPY_KIB / 2), ("WRITE_SIZE", [20.0, 20.0], COPY_KIB)):
        d = str(sandbox / counter)
        os.makedirs(os.path.join(d, "run"), exist_ok=True)
        rows = [("void fdtd::k_tblock_bt<5>(fdtd::InstDev const*, int)", v) for v in vals]
        rows += [("void fdtd::k_tblock_bb<5, false>(fdtd::InstDev const*, int)", 1e9),
                 ("__amd_rocclr_copyBuffer", copy_kib)]
        with open(os.path.join(d, "run", "pmc_counter_collection.csv"), "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"])
            for t, (k, v) in enumerate(rows):
                w.writerow([k, counter, v, 200 * t, 200 * t + 100])
        with open(d + ".log", "w") as f:
            f.write(json.dumps({"profile_pass": True, "workload": "broadband_healthy", "polarization": 1,
                                "bytes_per_cell": 40.0, "t_block": 5, "band_rows": 64, "lean_cells": 900,
                                "kernel_cells": 1000, "launches": 2, "copy_bytes": bench.COPY_BYTES}) + "\n")
    bench.derive_traffic(str(sandbox / "FETCH_SIZE"), str(sandbox / "WRITE_SIZE"))
    rec = json.load(open(sandbox / "profiles" / "traffic.json"))["broadband_healthy_te"]["K5_B64"]
    assert rec["counters"]["FETCH_SIZE"]["dispatches"] == 2
    assert rec["bytes_per_launch"] == pytest.approx((40.0 * 2.0 + 20.0) * 1024)
    assert rec["algorithmic_bytes_per_launch"] == 40.0 * 1000
