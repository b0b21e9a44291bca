"""bench.py's contract pieces that need no GPU: the one-GPU refusal, the
algorithmic bytes of each stage, and that measured traffic is reported only
for the kernel sources it was measured on."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_stage():
    w = dict(bench.WORKLOADS["lognormal-512"])
    npart, n3 = 9_997_050, 512 ** 3
    # float32, interlaced: two meshes of 4-byte reals
    assert bench.algorithmic_bytes("paint_z", w, npart) == 3 * 4 * npart + 2 * 4 * n3
    assert bench.algorithmic_bytes("fft_y", w, npart) == 2 * 2 * 4 * n3
    assert bench.algorithmic_bytes("xpass_bin", w, npart) == 2 * 4 * n3
    assert bench.algorithmic_bytes("bucket", w, npart) == 0
    w.update(dtype="f8", interlaced=False)
    assert bench.algorithmic_bytes("paint_z", w, npart) == 3 * 8 * npart + 8 * n3


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    for wl in ("lognormal-512", "zeldovich-1024"):
        path = os.path.join(ROOT, "profiles", f"traffic_{wl}.json")
        rec = json.load(open(path))
        assert set(rec["kernels"]) >= {"paint_z", "fft_y", "xpass_bin"}
        monkeypatch.setattr(bench, "source_hash", lambda: rec["source_hash"])
        got = bench.measured_traffic(wl, "paint_z")
        assert got == rec["kernels"]["paint_z"]["bytes_per_launch"] and got > 0
        monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
        assert bench.measured_traffic(wl, "paint_z") is None
    assert bench.measured_traffic("no-such-workload", "paint_z") is None


def test_source_hash_ignores_comments():
    code = "int f(int x) {  // the answer\n  /* more\n  words */ return x;\n}\n\n"
    assert bench._code_only(code) == "int f(int x) {\n   return x;\n}"
    assert bench._code_only(code) == bench._code_only(code.replace("the answer", "another"))


def test_oracle_errors_follow_the_float32_bar_definitions():
    # |dP|/|P| per bin, |dP_ell| / |P_0| for ell > 0, P(k, mu) relative
    import numpy as np

    want = {"modes": np.array([0, 4, 6]), "power": np.array([np.nan, 2.0, 4.0]),
            "poles": {0: np.array([np.nan, 2.0, 4.0]), 2: np.array([np.nan, 0.0, -1.0])},
            "modes2d": np.array([[0, 0], [2, 2]]), "power2d": np.array([[np.nan, np.nan],
                                                                       [1.0, 3.0]])}
    got = {"modes": np.array([0, 4, 6]), "power": np.array([np.nan, 2.0002, 4.0]),
           "poles": {0: np.array([np.nan, 2.0, 4.0]), 2: np.array([np.nan, 0.001, -1.0])},
           "power2d": np.array([[np.nan, np.nan], [1.0, 3.003]])}
    e = bench.oracle_errors(got, want)
    assert e["counts_equal"]
    assert abs(e["P"] - 1e-4) < 1e-12
    assert abs(e["P_2"] - 0.001 / 2.0) < 1e-12
    assert abs(e["P_kmu"] - 1e-3) < 1e-12
    got["modes"] = np.array([0, 4, 5])
    assert not bench.oracle_errors(got, want)["counts_equal"]


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, counter, value in rows:
            fh.write(f'{d},"{name}",{counter},{value}\n')


def test_traffic_summary_scales_counters_by_the_copy(tmp_path, monkeypatch):
    # a copy of 1 GiB whose FETCH_SIZE reads half its bytes (scale 2) and
    # WRITE_SIZE all of them; three calls of a pipeline whose paint fetches
    # 100 KiB (two dimension rows of 50) and writes 1000 KiB per call
    d = str(tmp_path)
    gib_kib = 1 << 20
    _counter_csv(os.path.join(d, "pmc_FETCH_SIZE_copy"),
                 [(1, "void at::fill_kernel", "FETCH_SIZE", 0),
                  (2, "void at::copy_kernel", "FETCH_SIZE", gib_kib // 2)])
    _counter_csv(os.path.join(d, "pmc_WRITE_SIZE_copy"),
                 [(1, "void at::fill_kernel", "WRITE_SIZE", gib_kib),
                  (2, "void at::copy_kernel", "WRITE_SIZE", gib_kib)])
    fetch, write = [], []
    for call in range(3):
        base = 10 * call
        fetch += [(base, "pk::k_paint_z<float, 512, 3, 2>(...)", "FETCH_SIZE", 50),
                  (base, "pk::k_paint_z<float, 512, 3, 2>(...)", "FETCH_SIZE", 50),
                  (base + 1, "pk::k_xpass_bin<float, 512>(...)", "FETCH_SIZE", 7)]
        write += [(base, "pk::k_paint_z<float, 512, 3, 2>(...)", "WRITE_SIZE", 1000),
                  (base + 1, "pk::k_xpass_bin<float, 512>(...)", "WRITE_SIZE", 1)]
    fetch.append((99, "pk::k_mode_tables(...)", "FETCH_SIZE", 12345))  # plan time: ignored
    _counter_csv(os.path.join(d, "pmc_FETCH_SIZE_lognormal-512"), fetch)
    _counter_csv(os.path.join(d, "pmc_WRITE_SIZE_lognormal-512"), write)
    monkeypatch.setattr(bench, "ROOT", d)
    os.makedirs(os.path.join(d, "profiles"))
    monkeypatch.setattr(bench, "source_hash", lambda: "f" * 16)
    path = bench.write_traffic("lognormal-512", d, 9_997_050)
    rec = json.load(open(path))
    assert rec["calls"] == 3 and rec["source_hash"] == "f" * 16
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    p = rec["kernels"]["paint_z"]
    assert p["fetch_bytes"] == 100 * 1024 * 2.0 and p["write_bytes"] == 1000 * 1024
    assert p["bytes_per_launch"] == p["fetch_bytes"] + p["write_bytes"]
    assert rec["kernels"]["xpass_bin"]["fetch_bytes"] == 7 * 1024 * 2.0
    assert rec["kernels"]["bucket"]["fetch_bytes"] == 0
