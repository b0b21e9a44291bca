"""GPU parity of the fused FFTPower path (pk_fftpower) against the float64
oracle on every k-bin, at the mesh sizes and windows the benchmarks run
(Sec. 3.3.1 painting, Sec. 3.3.2 interlacing and compensation, Sec. 3.4.1
binning).  The kernels that run depend on the mesh size, window and
precision, not on the number of particles, so the oracle's catalogs are
smaller than the benchmark catalogs:

* 1024^3 CIC interlaced, P_0 and P_2: a Zel'dovich lattice of 192^3
  particles in lattice order (the column-run route of the bucketing);
* 512^3 CIC interlaced, P(k, mu) with 5 mu bins and P_2: uniform particles
  in random order (the slab route);
* 256^3 TSC interlaced, P_0, P_2, P_4: a log-normal mock (the middle mesh of
  the batch of mocks).

At the full Zel'dovich catalog (512^3 particles on 1024^3), where the
oracle's complete run does not fit a test, every bin of the fused path is
compared with the stand-alone chain pk_paint (both shifts) -> pk_fft_r2c ->
pk_compensate -> pk_bin_power, which runs different kernels (the atomic
painter, the in-place three-pass transform, the separate binning).

Tolerance: the float32 bar, per bin |dP| / |P| <= 1e-5 and
|dP_ell| <= 1e-5 |P_0|; counts bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, synth
from tests.powercheck import check_power

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def fused(ctx, m, b, pos_d, npart):
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower(m, b, pos_d, None, npart, ws, res)
    out = ctx.pk_result_to_host(m, b, res)
    del ws, res
    torch.cuda.empty_cache()
    return out


def report(got, want, tag):
    ok = want["modes"] > 0
    rel = np.abs(got["power"][ok] / want["power"][ok] - 1)
    line = f"{tag}: {ok.sum()} bins, max |dP/P| {rel.max():.2e}"
    for ell, p in want["poles"].items():
        if ell:
            e = np.abs(got["poles"][ell][ok] - p[ok]) / np.abs(want["power"][ok])
            line += f", max |dP_{ell}|/|P_0| {e.max():.2e}"
    if "power2d" in want:
        ok2 = want["modes2d"] > 0
        line += f", max |dP(k,mu)/P| {np.abs(got['power2d'][ok2] / want['power2d'][ok2] - 1).max():.2e}"
    print(line, flush=True)


@pytest.mark.timeout(1200)
def test_fused_1024_cic_interlaced_every_bin(ctx):
    n, box = 1024, 2000.0
    pos = synth.zeldovich_lattice(192, box, synth.pk_zeldovich_c3, seed=3)
    print(f"\n1024^3 CIC interlaced: {len(pos)} particles (lattice order)", flush=True)
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    got = fused(ctx, m, b, dev(pos), len(pos))
    want = oracle.fftpower(pos.astype(np.float64), n, box, "cic", True, True, nmu=0,
                           poles=(0, 2))
    report(got, want, "1024^3 CIC")
    check_power(got, want, 1e-5, "1024^3 CIC interlaced")


@pytest.mark.timeout(600)
def test_fused_512_cic_interlaced_every_bin(ctx):
    n, box = 512, 1380.0
    pos = synth.uniform_catalog(2_000_000, box, seed=17).astype(np.float32)
    print(f"\n512^3 CIC interlaced: {len(pos)} particles (random order)", flush=True)
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 5, (0, 2), 2)
    got = fused(ctx, m, b, dev(pos), len(pos))
    want = oracle.fftpower(pos.astype(np.float64), n, box, "cic", True, True, nmu=5,
                           poles=(0, 2))
    report(got, want, "512^3 CIC")
    check_power(got, want, 1e-5, "512^3 CIC interlaced")


@pytest.mark.timeout(600)
def test_fused_256_tsc_interlaced_every_bin(ctx):
    n, box = 256, 1380.0
    pos = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 2e6 / n ** 3, seed=1001)
    print(f"\n256^3 TSC interlaced: {len(pos)} particles", flush=True)
    m = _lib.mesh_desc(n, box, "tsc", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2, 4), 2)
    got = fused(ctx, m, b, dev(pos), len(pos))
    want = oracle.fftpower(pos.astype(np.float64), n, box, "tsc", True, True, nmu=0,
                           poles=(0, 2, 4))
    report(got, want, "256^3 TSC")
    check_power(got, want, 1e-5, "256^3 TSC interlaced")


@pytest.mark.timeout(900)
def test_fused_1024_full_catalog_matches_standalone_chain(ctx):
    n, box = 1024, 2000.0
    pos = synth.zeldovich_lattice(512, box, synth.pk_zeldovich_c3, seed=3)
    npart = len(pos)
    print(f"\n1024^3 full catalog: {npart} particles", flush=True)
    pos_d = dev(pos)
    del pos
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    got = fused(ctx, m, b, pos_d, npart)
    a = torch.empty((n, n, n), dtype=torch.float32, device="cuda:0")
    bm = torch.empty_like(a)
    wsums = torch.empty(2, dtype=torch.float64, device="cuda:0")
    ctx.pk_paint(m, pos_d, None, npart, 0.0, a, wsums)
    ctx.pk_paint(m, pos_d, None, npart, 0.5, bm, None)
    ctx.pk_fft_r2c(m, a)
    ctx.pk_fft_r2c(m, bm)
    ctx.pk_compensate(m, a, bm)
    del bm
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power(m, b, a, res)
    res[-2:] = wsums
    chain = ctx.pk_result_to_host(m, b, res)
    del a
    torch.cuda.empty_cache()
    report(got, chain, "1024^3 fused vs chain")
    check_power(got, chain, 1e-5, "1024^3 fused vs stand-alone chain")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("compensated", [True, False])
def test_fused_1024_single_mesh_matches_standalone_chain(ctx, compensated):
    # one mesh (no interlacing), with and without the window compensation:
    # the x-pass takes one (tile, mesh) unit per tile
    n, box = 1024, 2000.0
    pos = synth.zeldovich_lattice(192, box, synth.pk_zeldovich_c3, seed=4)
    npart = len(pos)
    pos_d = dev(pos)
    m = _lib.mesh_desc(n, box, "cic", False, compensated, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    got = fused(ctx, m, b, pos_d, npart)
    a = torch.empty((n, n, n), dtype=torch.float32, device="cuda:0")
    wsums = torch.empty(2, dtype=torch.float64, device="cuda:0")
    ctx.pk_paint(m, pos_d, None, npart, 0.0, a, wsums)
    ctx.pk_fft_r2c(m, a)
    ctx.pk_compensate(m, a, None)
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power(m, b, a, res)
    res[-2:] = wsums
    chain = ctx.pk_result_to_host(m, b, res)
    del a
    torch.cuda.empty_cache()
    report(got, chain, f"1024^3 single mesh (compensated {compensated}) fused vs chain")
    check_power(got, chain, 1e-5, "1024^3 single mesh fused vs stand-alone chain")
