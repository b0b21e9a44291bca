#!/usr/bin/env python3
"""Benchmark of the FFTPower hot path on one MI355X.

One step = one pass of the whole path over one resident catalog: paint both
interlaced meshes, r2c FFT, interlace + compensate + bin, finalise (result
copied to the host).  Default workload (the one the headline metric is quoted
on): a Poisson-sampled log-normal mock of ~1e7 particles (P(k) =
2e4 k / (1 + (k / 0.02)^2)^1.4, L = 1380 Mpc/h), TSC interlaced onto a 512^3
float32 mesh, P(k, mu) with 5 mu bins and ell = 0, 2, 4 along z.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  ``value`` is meshes/s with the catalog resident in HBM;
``roofline`` prices the dominant kernel's algorithmic bytes against 8 TB/s
using HIP events recorded by the library on its stream; ``cpu_baseline`` times
the CPU float64 oracle on a bounded sample of the same workload.
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mparticles/s painted + P(k) meshes/s at 512³; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "lognormal-512": dict(n=512, box=1380.0, window="tsc", interlaced=True, dtype="f4",
                          nmu=5, poles=(0, 2, 4), kind="lognormal", seed=2),
    "zeldovich-1024": dict(n=1024, box=2000.0, window="cic", interlaced=True, dtype="f4",
                           nmu=0, poles=(0, 2), kind="zeldovich", ngrid=512, seed=3),
    "uniform-64-fp64": dict(n=64, box=1000.0, window="cic", interlaced=False, dtype="f8",
                            nmu=0, poles=(), kind="uniform", npart=10_000, seed=1),
}


# Many uneven mocks in one batch (the paper's repeated-analysis use case,
# Sec. 6): log-normal catalogs with N_i = round(10^U(5, 7)) particles on
# 128^3 / 256^3 / 512^3 meshes (by index), TSC interlaced float32, P(k) with
# ell = 0, 2, 4; catalogs drawn on the device (untimed).
BATCH = dict(count=256, box=1380.0, meshes=(128, 256, 512), seed=1000, lanes=8,
             window="tsc", poles=(0, 2, 4))


# Survey multipoles with a varying line of sight (ConvolvedFFTPower): a
# log-normal catalog (0.05 per cell on 512^3, ~6.7M in the box) and 10x as
# many uniform randoms, both cut to the shell 0.3 L <= |x - o| < 1.2 L around
# an observer at (L/2, L/2, -L/4); TSC, compensated, float32, ell = 0, 2, 4
# (1 + 5 + 9 harmonic paintings and FFTs per call).
SURVEY = dict(n=512, box=2000.0, window="tsc", nbar_cell=0.05, rand_factor=10.0, seed=5,
              observer=(0.5, 0.5, -0.25), shell=(0.3, 1.2), poles=(0, 2, 4))


# Serving: requests arriving as a Poisson process; per request a uniform or
# log-normal catalog (50/50), N_p log-uniform in [1e5, 5e7], mesh 128^3 ..
# 1024^3, CIC or TSC, interlacing on or off, float32.  Catalogs are drawn on
# the device before the run (untimed, log-normal on a min(N, 512)^3 grid).
SERVE = dict(count=120, qps=(10.0, 40.0, 160.0, 640.0), seed=5, lanes=8, box=1380.0,
             meshes=(128, 256, 512, 1024), np_range=(1e5, 5e7), reserve_gib=8.0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_catalog(w):
    import numpy as np

    from paper_1712_05834_amd import synth

    nd = np.float32 if w["dtype"] == "f4" else np.float64
    if w["kind"] == "lognormal":
        n = w["n"]
        return synth.lognormal_catalog(n, w["box"], synth.pk_lognormal_c2, 1e7 / n ** 3,
                                       seed=w["seed"], dtype=nd)
    if w["kind"] == "zeldovich":
        return synth.zeldovich_lattice(w["ngrid"], w["box"], synth.pk_zeldovich_c3,
                                       seed=w["seed"], dtype=nd)
    return synth.uniform_catalog(w["npart"], w["box"], seed=w["seed"], dtype=nd)


def algorithmic_bytes(stage, w, npart):
    """Compulsory HBM bytes of one launch of a stage: each input read once and
    each output written once: painting reads 3e bytes per particle and writes
    e per cell and mesh, each FFT pass reads and writes e per real point and
    mesh, the binning reads e per real point and mesh.  The bucketing
    pass only reorders the catalog, so it has none; the fused paint + z-pass
    consumes the catalog and writes the z-transformed meshes."""
    es = 4 if w["dtype"] == "f4" else 8
    n3 = w["n"] ** 3
    m = 2 if w["interlaced"] else 1
    return {
        "paint_z": 3 * es * npart + m * es * n3,   # positions in, packed rows out
        "fft_y": m * 2 * es * n3,                  # packed rows in and out
        "xpass_bin": m * es * n3,                  # spectra in, ~10 KB of sums out
        "plane_bin": m * 2 * es * w["n"] ** 2,
    }.get(stage, 0)


def _code_only(text):
    """The source with // and /* */ comments and blank lines removed (the
    kernels' sources contain no string literals with comment markers)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def source_hash():
    """Hash of the kernel sources' code (comments and blank lines ignored), so
    that measured traffic stays attached to the code it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1712_05834_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(f.encode() + _code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    there are none or the kernels changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# Kernels of each pk_fftpower stage, by name without template arguments
# (plan-time tables and copies are not part of a call).
STAGE_KERNELS = {
    "bucket": ("k_fill_zero", "k_order_probe", "k_bucket_count", "k_weight_sums", "k_scan_blocks",
               "k_scan_sums", "k_scan_final", "k_slab_columns", "k_bucket_scatter"),
    "paint_z": ("k_paint_z",),
    "fft_y": ("k_fft_y_relayout",),
    "xpass_bin": ("k_xpass_bin",),
    "plane_bin": ("k_plane_bin",),
    "reduce": ("k_reduce",),
}


def _counter_totals(directory, counter):
    """{kernel name: [per-dispatch sums of counter]} from the rocprofv3 CSVs
    under directory (rows of one dispatch summed over their dimensions)."""
    import csv
    import glob

    per = {}
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = re.sub(r"\(.*\)$", "", re.sub(r"^void ", "", row.get("Kernel_Name", "")))
                key = (name, row.get("Dispatch_Id"))
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def write_traffic(workload, directory, npart):
    """profiles/traffic_<workload>.json from four rocprofv3 --pmc runs under
    directory: pmc_FETCH_SIZE_<workload>, pmc_WRITE_SIZE_<workload> (the bench
    with --steps 2 --warmup 1) and pmc_FETCH_SIZE_copy, pmc_WRITE_SIZE_copy
    (--calibrate-copy 1024).  The counters, in KiB per dispatch, are scaled
    by what they read for a plain copy of known size."""
    w = WORKLOADS[workload]
    copy_bytes = 1024 << 20
    cal = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [v for vs in _counter_totals(os.path.join(directory, f"pmc_{counter}_copy"),
                                            counter).values() for v in vs]
        kib = max(vals)  # the copy kernel's dispatches (the largest ones)
        cal[counter] = (kib, copy_bytes / (kib * 1024.0))
    stages = {}
    totals = {c: _counter_totals(os.path.join(directory, f"pmc_{c}_{workload}"), c)
              for c in ("FETCH_SIZE", "WRITE_SIZE")}
    calls = len(next((v for k, v in totals["FETCH_SIZE"].items() if "k_xpass_bin" in k), []))
    for stage, prefixes in STAGE_KERNELS.items():
        names = sorted({k for c in totals for k in totals[c]
                        if re.sub(r"<.*", "", k) in {"pk::" + p for p in prefixes}})
        b = {}
        for c, key in (("FETCH_SIZE", "fetch_bytes"), ("WRITE_SIZE", "write_bytes")):
            kib = sum(sum(totals[c].get(k, [])) for k in names)
            b[key] = kib * 1024.0 * cal[c][1] / max(calls, 1)
        alg = algorithmic_bytes(stage, w, npart)
        per = b["fetch_bytes"] + b["write_bytes"]
        stages[stage] = {"kernels": names, **b, "bytes_per_launch": per,
                         "algorithmic_bytes": alg,
                         "ratio_to_algorithmic": per / alg if alg else None}
    base = "python3 bench.py --workload {wl} --steps 2 --warmup 1 --no-cpu-baseline --no-latency"
    rec = {
        "workload": workload, "npart": npart, "source_hash": source_hash(), "calls": calls,
        "commands": [f"rocprofv3 --pmc {c} -f csv -d gpurun_out/pmc_{c}_{workload} -o run -- "
                     + base.format(wl=workload) for c in ("FETCH_SIZE", "WRITE_SIZE")] +
                    [f"rocprofv3 --pmc {c} -f csv -d gpurun_out/pmc_{c}_copy -o run -- "
                     "python3 bench.py --calibrate-copy 1024" for c in ("FETCH_SIZE", "WRITE_SIZE")],
        "calibration": {"copy_bytes": copy_bytes,
                        "fetch_kib_reported": cal["FETCH_SIZE"][0], "fetch_scale": cal["FETCH_SIZE"][1],
                        "write_kib_reported": cal["WRITE_SIZE"][0], "write_scale": cal["WRITE_SIZE"][1]},
        "note": "bytes per pk_fftpower call (all launches of the stage), scaled by the copy "
                "calibration",
        "kernels": stages,
    }
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return path


def request_latency(ctx, m, b, pos, npart, step_ms, count=60, lanes=2):
    """p50 / p99 latency (arrival to result on the host) of `count` requests
    of the timed workload arriving as a Poisson process at half the rate one
    GPU sustains (1 / step_ms), served on `lanes` lanes of the context; the
    catalog stays resident, each request gets its own workspace."""
    import torch

    from paper_1712_05834_amd import synth
    from paper_1712_05834_amd.serve import (LibpkBackend, Request, Server, latency_stats,
                                            poisson_arrivals)

    qps = 0.5 * 1e3 / step_ms
    backend = LibpkBackend(ctx, lanes)
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - 8 * 2 ** 30)
    Server(backend, budget).run([Request(-1, 0.0, m, b, pos, npart)])  # lanes warmed up
    arrivals = poisson_arrivals(count, qps, synth.rng_for(77))
    reqs = [Request(i, a, m, b, pos, npart) for i, a in enumerate(arrivals)]
    st = latency_stats(Server(backend, budget).run(reqs))
    st.update(qps=qps, lanes=lanes)
    return st


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def run_fft_reference(args):
    """The stand-alone hand-written r2c (pk_fft_r2c: z, y and x passes in
    place on the packed layout) timed beside rocFFT's r2c (torch.fft.rfftn,
    out of place) on the same float32 meshes: a reference point only, the
    power-spectrum path does not use it."""
    import numpy as np
    import torch

    from paper_1712_05834_amd import _lib

    dev = torch.device("cuda:0")
    ctx = _lib.Context(0)
    out = {"metric": "r2c 3-D FFT time, hand-written vs rocFFT (torch.fft.rfftn)",
           "unit": "ms", "dtype": "f32", "data": "synthetic (standard normal mesh)", "sizes": []}
    for n in (256, 512, 1024):
        src = torch.randn((n, n, n), dtype=torch.float32, device=dev,
                          generator=torch.Generator(device=dev).manual_seed(n))
        work = torch.empty_like(src)
        m = _lib.mesh_desc(n, 1000.0, "cic", False, True, "f4")
        ours, roc = [], []
        for rep in range(args.warmup + args.steps):
            work.copy_(src)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.pk_fft_r2c(m, work)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            spec = torch.fft.rfftn(src)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            del spec
            if rep >= args.warmup:
                ours.append(t1 - t0)
                roc.append(t2 - t1)
        row = {"n": n, "hand_written_ms": 1e3 * float(np.median(ours)),
               "rocfft_ms": 1e3 * float(np.median(roc))}
        row["rocfft_over_hand_written"] = row["rocfft_ms"] / row["hand_written_ms"]
        log(f"r2c {n}^3: hand-written {row['hand_written_ms']:.3f} ms, "
            f"rocFFT {row['rocfft_ms']:.3f} ms (median of {args.steps})")
        out["sizes"].append(row)
        del src, work
        torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps(out))


def oracle_errors(got, want):
    """Largest per-bin error of a GPU FFTPower result against the float64
    oracle's, on the definitions of the float32 bar: |dP| / |P| for P(k) and
    P(k, mu), |dP_ell| / |P_0| for ell > 0 (P_ell crosses zero); counts must
    agree exactly."""
    import numpy as np

    ok = want["modes"] > 0
    out = {"counts_equal": bool(np.array_equal(got["modes"], want["modes"])),
           "P": float(np.max(np.abs(got["power"][ok] / want["power"][ok] - 1)))}
    for ell, p in want["poles"].items():
        if ell:
            out[f"P_{ell}"] = float(np.max(np.abs(got["poles"][ell][ok] - p[ok])
                                           / np.abs(want["power"][ok])))
    if "power2d" in want:
        ok2 = want["modes2d"] > 0
        out["P_kmu"] = float(np.max(np.abs(got["power2d"][ok2] / want["power2d"][ok2] - 1)))
    return out


def cpu_baseline(w, pos, frac):
    """The CPU float64 oracle on a bounded sample of the catalog: painting of
    both meshes, the full r2c of each mesh and the full binning, each stage
    timed; the painting is scaled by 1 / frac to the whole catalog.  Returns
    the baseline entry, the oracle's result for the sample and the sample
    itself (to run the GPU path on the same particles)."""
    import numpy as np

    import oracle
    from oracle.paint import WINDOW_ORDER

    n, box, order = w["n"], w["box"], WINDOW_ORDER[w["window"]]
    sub = pos[: max(1, int(len(pos) * frac))]
    sub64 = sub.astype(np.float64)
    t0 = time.perf_counter()
    ma = oracle.paint_mesh(sub64, n, box, order)
    mb = oracle.paint_mesh(sub64, n, box, order, shift_cells=0.5) if w["interlaced"] else None
    t_paint = time.perf_counter() - t0
    t0 = time.perf_counter()
    ca = oracle.r2c(ma)
    del ma
    cb = oracle.r2c(mb) if mb is not None else None
    del mb
    t_fft = time.perf_counter() - t0
    t0 = time.perf_counter()
    want = oracle.fftpower_from_spectra(ca, cb, n, box, order, True, float(len(sub)),
                                        float(len(sub)), len(sub), nmu=w["nmu"],
                                        poles=w["poles"])
    t_bin = time.perf_counter() - t0
    del ca, cb
    per_mesh = t_paint / frac + t_fft + t_bin
    scaled = "" if frac >= 1 else f", scaled x{1 / frac:g}"
    entry = {
        "value": 1.0 / per_mesh,
        "unit": "meshes/s",
        "cores": os.cpu_count(),
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": (f"float64 oracle on this host: painting of {len(sub)} of {len(pos)} "
                   f"particles onto {'both meshes' if w['interlaced'] else 'the mesh'} "
                   f"({t_paint:.1f} s, single thread{scaled}), full r2c "
                   f"({t_fft:.1f} s, scipy workers={os.cpu_count()}) and full binning "
                   f"({t_bin:.1f} s, single thread) of one {n}^3 mesh"),
    }
    return entry, want, sub


def oracle_on_items(items, unit):
    """cpu_baseline of the batch and serving workloads: the float64 oracle on
    a few of the catalogs, timed, and the GPU results of those catalogs
    against it.  items: (label, positions on the host, nmesh, boxsize,
    window, interlaced, poles, GPU result)."""
    import numpy as np

    import oracle

    t_total, errs = 0.0, []
    for label, pos, n, box, window, inter, poles, got in items:
        t0 = time.perf_counter()
        want = oracle.fftpower(pos.astype(np.float64), n, box, window, inter, True, nmu=0,
                               poles=poles)
        t_total += time.perf_counter() - t0
        e = oracle_errors(got, want)
        e["catalog"] = label
        errs.append(e)
    worst = {"P": max(e["P"] for e in errs), "counts_equal": all(e["counts_equal"] for e in errs)}
    for key in {k for e in errs for k in e if k.startswith("P_")}:
        worst[key] = max(e.get(key, 0.0) for e in errs)
    entry = {"value": len(items) / t_total, "unit": unit, "cores": os.cpu_count(),
             "cpu": cpu_model(), "kind": "oracle",
             "sample": (f"float64 oracle on this host ({os.cpu_count()} cores for the r2c, "
                        f"one for painting and binning) on {len(items)} of the catalogs: "
                        + "; ".join(e["catalog"] for e in errs) + f" ({t_total:.1f} s)")}
    return entry, {"worst": worst, "per_catalog": errs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal-512",
                    choices=sorted(WORKLOADS) + ["batch-mocks", "serve", "survey-512",
                                                 "fft-reference"])
    ap.add_argument("--mocks", type=int, default=BATCH["count"],
                    help="number of mocks of the batch-mocks workload")
    ap.add_argument("--lanes", type=int, default=BATCH["lanes"],
                    help="concurrent lanes of the batch-mocks workload")
    ap.add_argument("--autotune", action="store_true",
                    help="tune pk_fftpower's launch choices on the first warm-up call (the "
                         "line then reports the chosen settings)")
    ap.add_argument("--graph", action="store_true",
                    help="batch-mocks: capture the whole batch into one HIP graph and time its "
                         "replays instead of enqueueing it call by call")
    ap.add_argument("--batch-meshes", default=None,
                    help="batch-mocks: keep only the mocks on these mesh sizes (comma list), to "
                         "time parts of the batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the request-latency leg (p50 / p99 of requests of the workload "
                         "arriving at half the sustained rate)")
    ap.add_argument("--shuffle", action="store_true",
                    help="permute the catalog (seeded) before timing: a catalog in no "
                         "particular order instead of the generator's cell order")
    ap.add_argument("--cpu-sample", type=float, default=None,
                    help="fraction of the catalog the oracle paints for cpu_baseline "
                         "(default: the whole catalog at 512^3 and below, 3%% at 1024^3)")
    ap.add_argument("--traffic-from", default=None, metavar="DIR",
                    help="write profiles/traffic_<workload>.json from the rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE runs under DIR (see write_traffic) and exit; "
                         "needs --npart, no GPU")
    ap.add_argument("--npart", type=int, default=0,
                    help="particles of the workload's catalog (for --traffic-from)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) and exit: the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.traffic_from:
        print(write_traffic(args.workload, args.traffic_from, args.npart))
        return
    if args.calibrate_copy:
        import torch

        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(each mesh is processed on a single MI355X; sharding one mesh across GPUs is "
              "not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1712_05834_amd import _lib

    if args.workload == "batch-mocks":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "survey-512":
        run_survey(args)
        return
    if args.workload == "fft-reference":
        run_fft_reference(args)
        return
    w = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    pos_host = make_catalog(w)
    npart = len(pos_host)
    if args.shuffle:
        pos_host = pos_host[np.random.default_rng(12345).permutation(npart)]
    log(f"workload {args.workload}: {npart} particles generated in "
        f"{time.perf_counter() - t0:.1f} s" + (" (shuffled)" if args.shuffle else ""))

    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_host).to(dev)
    ctx = _lib.Context(0)
    m = _lib.mesh_desc(w["n"], w["box"], w["window"], w["interlaced"], True, w["dtype"])
    b = _lib.bin_desc(w["n"] // 2, 0.0, 1.0, w["nmu"], w["poles"], 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device=dev)
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device=dev)

    def step():
        ctx.pk_fftpower(m, b, pos, None, npart, ws, res)
        return ctx.pk_result_to_host(m, b, res)

    if args.autotune:
        ctx.pk_ctx_set_autotune(1)
    for _ in range(max(args.warmup, 1 if args.autotune else 0)):
        step()
    torch.cuda.synchronize()
    if args.autotune:
        log(f"tuned: {ctx.tune_table()}")
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")

    ctx.pk_ctx_set_timing(True)
    stage_ms = {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_ends = []
    for _ in range(args.steps):
        out = step()  # ends with the result on the host (synchronised)
        step_ends.append(time.perf_counter())
        for k, v in ctx.pk_ctx_stage_times().items():
            stage_ms.setdefault(k, []).append(v)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    step_ms = np.diff([t_start] + step_ends) * 1e3
    ctx.pk_ctx_set_timing(False)

    ms_per_step = 1e3 * elapsed / args.steps
    mean_ms = {k: float(np.mean(v)) for k, v in stage_ms.items()}
    log("stage means (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in mean_ms.items()))
    paint_ms = mean_ms.get("bucket", 0.0) + mean_ms.get("paint_z", 0.0)
    dominant = max((k for k in mean_ms if algorithmic_bytes(k, w, npart) > 0),
                   key=lambda k: mean_ms[k])
    nbytes = algorithmic_bytes(dominant, w, npart)
    achieved = nbytes / (mean_ms[dominant] * 1e-3) / 1e9
    total_bytes = sum(algorithmic_bytes(k, w, npart) for k in mean_ms)
    assert np.isfinite(out["power"][1:]).all(), "non-finite power"

    line = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "meshes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (paint, FFT) + f64 (bin sums)" if w["dtype"] == "f4" else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "nmesh": w["n"], "boxsize": w["box"], "window": w["window"],
            "interlaced": w["interlaced"], "npart": npart, "nmu": w["nmu"],
            "poles": list(w["poles"]), "los": "z",
            "order": "shuffled" if args.shuffle else "as generated",
        },
        "tuned": ctx.tune_table() if args.autotune else None,
        "mparticles_per_s_painted": npart / (paint_ms * 1e-3) / 1e6 if paint_ms > 0 else None,
        "stage_ms": mean_ms,
        "end_to_end_hbm_frac": total_bytes / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "roofline": {
            "bound": "hbm",
            "kernel": dominant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if args.shuffle else measured_traffic(args.workload, dominant),
        },
        "cpu_baseline": None,
        "latency": None,
    }
    if not args.no_latency:
        line["latency"] = request_latency(ctx, m, b, pos, npart, ms_per_step)
        log(f"request latency at {line['latency']['qps']:.0f} QPS: p50 "
            f"{line['latency']['p50_ms']:.2f} ms, p99 {line['latency']['p99_ms']:.2f} ms")
    if not args.no_cpu_baseline:
        frac = args.cpu_sample if args.cpu_sample else (1.0 if w["n"] <= 512 else 0.03)
        log(f"timing the CPU oracle on {frac:g} of the catalog")
        line["cpu_baseline"], want, sub = cpu_baseline(w, pos_host, frac)
        if len(sub) == npart:
            got, basis = out, "the timed run's result, whole catalog"
        else:
            # the GPU path once more, untimed, on the oracle's sample
            sub_d = torch.from_numpy(np.ascontiguousarray(sub)).to(dev)
            ws_s = torch.empty(_lib.workspace_bytes(m, b, len(sub)), dtype=torch.uint8,
                               device=dev)
            ctx.pk_fftpower(m, b, sub_d, None, len(sub), ws_s, res)
            got = ctx.pk_result_to_host(m, b, res)
            basis = f"the same path on the oracle's sample of {len(sub)} particles"
        err = oracle_errors(got, want)
        err["basis"] = basis
        line["max_rel_err_vs_oracle"] = err
        log("error against the float64 oracle: " + ", ".join(
            f"{k} {v:.2e}" for k, v in err.items() if isinstance(v, float)))
    print(json.dumps(line), flush=True)


def run_batch(args):
    """batch-mocks: one step = pk_fftpower_batch over all mocks + every result
    to the host.  value = mocks/s.  Also reports, untimed, the float32 result
    against the float64 path per mock."""
    import numpy as np
    import torch

    from paper_1712_05834_amd import _lib, synth

    dev = torch.device("cuda:0")
    sizes = synth.mock_batch_sizes(args.mocks, BATCH["seed"], BATCH["meshes"])
    keep = None if not args.batch_meshes else {int(v) for v in args.batch_meshes.split(",")}
    t0 = time.perf_counter()
    pos, ms, bs, res = [], [], [], []
    for i, (target, n) in enumerate(sizes):
        if keep is not None and n not in keep:
            continue
        p = synth.lognormal_catalog_device(n, BATCH["box"], synth.pk_lognormal_c2, target / n ** 3,
                                           seed=BATCH["seed"] + i, device=dev)
        pos.append(p)
        ms.append(_lib.mesh_desc(n, BATCH["box"], BATCH["window"], True, True, "f4"))
        bs.append(_lib.bin_desc(n // 2, 0.0, 1.0, 0, BATCH["poles"], 2))
        res.append(torch.empty(_lib.result_doubles(bs[-1]), dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    npart = [int(p.shape[0]) for p in pos]
    log(f"batch-mocks: {len(pos)} mocks, {sum(npart)} particles drawn on the device in "
        f"{time.perf_counter() - t0:.1f} s")
    # a stream of our own: graph capture is refused on the legacy default stream
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = _lib.Context(0, stream)
    ctx.pk_ctx_set_lanes(args.lanes)
    need = max(_lib.workspace_bytes(m, b, n) for m, b, n in zip(ms, bs, npart))
    lane_ws = [torch.empty(need, dtype=torch.uint8, device=dev) for _ in range(args.lanes)]
    log(f"{args.lanes} lanes, {need / 2**30:.2f} GiB of workspace each")

    def eager_step():
        ctx.pk_fftpower_batch(ms, bs, pos, [None] * len(pos), npart, lane_ws, res)
        return [ctx.pk_result_to_host(m, b, r) for m, b, r in zip(ms, bs, res)]

    step = eager_step
    graph = None
    if args.graph:
        eager_step()  # tables built
        t_cap = time.perf_counter()
        graph = ctx.pk_fftpower_batch_graph(ms, bs, pos, [None] * len(pos), npart, lane_ws, res)
        log(f"batch captured into one HIP graph of {graph.nodes} nodes in "
            f"{1e3 * (time.perf_counter() - t_cap):.1f} ms")

        def step():
            graph.launch()
            return [ctx.pk_result_to_host(m, b, r) for m, b, r in zip(ms, bs, res)]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    # algorithmic bytes of the batch (same per-stage figures as one mock)
    total = 0
    for (target, n), npt in zip(sizes, npart):
        wl = dict(dtype="f4", n=n, interlaced=True)
        total += sum(algorithmic_bytes(st, wl, npt) for st in ("paint_z", "fft_y", "xpass_bin",
                                                               "plane_bin"))
    achieved = total / (ms_per_step * 1e-3) / 1e9
    # float32 against float64, per mock (untimed)
    errs = []
    for i in range(len(pos)):
        m8 = _lib.mesh_desc(ms[i].nmesh, BATCH["box"], BATCH["window"], True, True, "f8")
        p8 = pos[i].double()
        ws8 = torch.empty(_lib.workspace_bytes(m8, bs[i], npart[i]), dtype=torch.uint8, device=dev)
        r8 = torch.empty_like(res[i])
        ctx.pk_fftpower(m8, bs[i], p8, None, npart[i], ws8, r8)
        want = ctx.pk_result_to_host(m8, bs[i], r8)
        ok = want["modes"] > 0
        errs.append(float(np.max(np.abs(out[i]["power"][ok] / want["power"][ok] - 1))))
        del ws8, p8
    line = {
        "metric": "mocks/s (FFTPower of many uneven log-normal mocks)",
        "value": len(pos) * 1e3 / ms_per_step,
        "unit": "mocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (paint, FFT) + f64 (bin sums)",
        "data": "synthetic (device-drawn log-normal mocks)",
        "config": {"workload": "batch-mocks", "mocks": len(pos), "lanes": args.lanes,
                   "graph": bool(args.graph),
                   "batch_meshes": sorted(keep) if keep else list(BATCH["meshes"]),
                   "meshes": list(BATCH["meshes"]), "npart_total": sum(npart),
                   "window": BATCH["window"], "interlaced": True,
                   "poles": list(BATCH["poles"])},
        "roofline": {"bound": "hbm", "kernel": "whole batch", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
        "fp32_vs_fp64_max_rel_err": {"max": max(errs), "median": float(np.median(errs))},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the smallest catalog of each mesh size, against the float64 oracle
        items = []
        for nm in BATCH["meshes"]:
            idx = [i for i in range(len(pos)) if ms[i].nmesh == nm]
            if not idx:
                continue
            i = min(idx, key=lambda j: npart[j])
            items.append((f"mock {i}: {npart[i]} particles on {nm}^3", pos[i].cpu().numpy(), nm,
                          BATCH["box"], BATCH["window"], True, BATCH["poles"], out[i]))
        log(f"float64 oracle on {len(items)} mocks")
        line["cpu_baseline"], line["max_rel_err_vs_oracle"] = oracle_on_items(items, "mocks/s")
    print(json.dumps(line), flush=True)


def run_survey(args):
    """survey-512: one step = pk_convolved_power + the multipoles on the host.
    value = survey multipole sets per second."""
    import numpy as np
    import torch

    from paper_1712_05834_amd import _lib, synth

    w = SURVEY
    box, n = w["box"], w["n"]
    obs = np.array(w["observer"]) * box
    t0 = time.perf_counter()
    data, rand = synth.survey_catalog(n, box, synth.pk_lognormal_c2, w["nbar_cell"], w["seed"],
                                      obs, w["shell"][0] * box, w["shell"][1] * box,
                                      w["rand_factor"], dtype=np.float32)
    log(f"survey: {len(data)} data, {len(rand)} randoms in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    d, r = torch.from_numpy(data).to(dev), torch.from_numpy(rand).to(dev)
    ctx = _lib.Context(0)
    m = _lib.mesh_desc(n, box, w["window"], False, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, w["poles"], 2)
    ws = torch.empty(_lib.convolved_workspace_bytes(m, b, len(data), len(rand)),
                     dtype=torch.uint8, device=dev)
    res = torch.empty(_lib.convolved_doubles(b), dtype=torch.float64, device=dev)
    norm = float(len(data)) ** 2 / box ** 3

    def step():
        ctx.pk_convolved_power(m, b, obs, d, None, len(data), r, None, len(rand), ws, res)
        return ctx.pk_convolved_to_host(m, b, norm, res)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    t_start = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    assert np.isfinite(out["poles"][0][1:]).all(), "non-finite multipoles"
    ms = 1e3 * elapsed / args.steps
    harmonics = sum(2 * ell + 1 for ell in set(w["poles"]) | {0})
    print(json.dumps({
        "metric": "survey multipole sets (P_0, P_2, P_4 with a varying line of sight) per second",
        "value": 1e3 / ms, "unit": "sets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (paint, FFT, fields) + f64 (bin sums)",
        "data": "synthetic",
        "config": {"workload": "survey-512", "nmesh": n, "boxsize": box,
                   "window": w["window"], "n_data": len(data), "n_rand": len(rand),
                   "poles": list(w["poles"]), "harmonics": harmonics},
        "ms_per_harmonic": ms / harmonics,
        "mparticles_per_s_painted": harmonics * (len(data) + len(rand)) / (ms * 1e-3) / 1e6,
    }), flush=True)


def run_serve(args):
    """serve: the same request pool served at several Poisson arrival rates.
    value = requests/s sustained at the highest rate; p50 / p99 latency
    (result on the host - arrival) per rate."""
    import numpy as np
    import torch

    from paper_1712_05834_amd import _lib, synth
    from paper_1712_05834_amd.serve import LibpkBackend, Request, Server, latency_stats
    from paper_1712_05834_amd.serve import poisson_arrivals

    dev = torch.device("cuda:0")
    rng = synth.rng_for(SERVE["seed"])
    lo, hi = np.log10(SERVE["np_range"][0]), np.log10(SERVE["np_range"][1])
    pool = []
    t0 = time.perf_counter()
    for i in range(SERVE["count"]):
        kind = "lognormal" if rng.uniform() < 0.5 else "uniform"
        target = int(round(10 ** rng.uniform(lo, hi)))
        n = int(SERVE["meshes"][rng.integers(len(SERVE["meshes"]))])
        window = "tsc" if rng.uniform() < 0.5 else "cic"
        inter = bool(rng.uniform() < 0.5)
        if kind == "lognormal":
            g = min(n, 512)
            pos = synth.lognormal_catalog_device(g, SERVE["box"], synth.pk_lognormal_c2,
                                                 target / g ** 3, seed=SERVE["seed"] * 1000 + i,
                                                 device=dev)
        else:
            gen = torch.Generator(device=dev)
            gen.manual_seed(SERVE["seed"] * 1000 + i)
            pos = torch.rand((target, 3), generator=gen, device=dev,
                             dtype=torch.float64) * SERVE["box"]
            pos = pos.to(torch.float32)
            pos[pos >= SERVE["box"]] = 0
        m = _lib.mesh_desc(n, SERVE["box"], window, inter, True, "f4")
        b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
        pool.append((m, b, pos))
    torch.cuda.synchronize()
    log(f"serve: {len(pool)} catalogs ({sum(p[2].shape[0] for p in pool)} particles) drawn on "
        f"the device in {time.perf_counter() - t0:.1f} s")
    ctx = _lib.Context(0)
    backend = LibpkBackend(ctx, SERVE["lanes"])
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - SERVE["reserve_gib"] * 2 ** 30)
    log(f"{SERVE['lanes']} lanes, admission budget {budget / 2**30:.0f} GiB")
    # warm-up: every mesh size and binning once (plan-time tables)
    warm = [Request(-1 - i, 0.0, m, b, p, p.shape[0]) for i, (m, b, p) in enumerate(pool[:8])]
    Server(backend, budget).run(warm)
    levels = []
    for qps in SERVE["qps"]:
        arr = poisson_arrivals(len(pool), qps, synth.rng_for(SERVE["seed"] + int(qps)))
        reqs = [Request(i, a, m, b, p, p.shape[0]) for i, (a, (m, b, p)) in enumerate(zip(arr, pool))]
        served = Server(backend, budget).run(reqs)
        st = latency_stats(served)
        st["qps"] = qps
        levels.append(st)
        log(f"qps {qps:g}: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
            f"{st['throughput_rps']:.1f} req/s")
    top = levels[-1]
    # float32 against the float64 path, per request of the last level (untimed)
    errs = []
    for r in served:
        m8 = _lib.mesh_desc(r.mesh.nmesh, r.mesh.boxsize, r.mesh.window, r.mesh.interlaced,
                            r.mesh.compensated, "f8")
        p8 = r.pos.double()
        ws8 = torch.empty(_lib.workspace_bytes(m8, r.bins, r.npart), dtype=torch.uint8,
                          device=dev)
        r8 = torch.empty(_lib.result_doubles(r.bins), dtype=torch.float64, device=dev)
        ctx.pk_fftpower(m8, r.bins, p8, None, r.npart, ws8, r8)
        want = ctx.pk_result_to_host(m8, r.bins, r8)
        ok = want["modes"] > 0
        errs.append(float(np.max(np.abs(r.result["power"][ok] / want["power"][ok] - 1))))
        del ws8, p8, r8
    log(f"float32 against float64 over {len(errs)} requests: max rel err {max(errs):.2e}, "
        f"median {np.median(errs):.2e}")
    line = {
        "metric": "p50/p99 request latency and sustained requests/s (FFTPower serving)",
        "value": top["throughput_rps"],
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": len(pool),
        "warmup": len(warm),
        "ms_per_step": 1e3 / top["throughput_rps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (paint, FFT) + f64 (bin sums)",
        "data": "synthetic (device-drawn uniform and log-normal catalogs)",
        "config": {"workload": "serve", "requests_per_level": len(pool),
                   "lanes": SERVE["lanes"], "meshes": list(SERVE["meshes"]),
                   "np_range": list(SERVE["np_range"]), "qps": list(SERVE["qps"])},
        "latency": levels,
        "fp32_vs_fp64_max_rel_err": {"max": max(errs), "median": float(np.median(errs))},
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the smallest request of each mesh size up to 512^3 (and each kind of
        # window and interlacing that occurs among them), against the oracle
        items, seen = [], set()
        for r in sorted(served, key=lambda q: q.npart):
            key = (r.mesh.nmesh, r.mesh.window, r.mesh.interlaced)
            if r.mesh.nmesh > 512 or r.npart > 3_000_000 or key in seen:
                continue
            seen.add(key)
            win = {2: "cic", 3: "tsc", 4: "pcs"}[r.mesh.window]
            items.append((f"request {r.rid}: {r.npart} particles, {r.mesh.nmesh}^3 {win}"
                          f"{' interlaced' if r.mesh.interlaced else ''}", r.pos.cpu().numpy(),
                          r.mesh.nmesh, r.mesh.boxsize, win, bool(r.mesh.interlaced), (0, 2),
                          r.result))
            if len(items) == 6:
                break
        log(f"float64 oracle on {len(items)} requests")
        line["cpu_baseline"], line["max_rel_err_vs_oracle"] = oracle_on_items(items, "requests/s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
