"""GPU parity at the benchmark workloads' full sizes.

* Log-normal mock, 512^3, TSC interlaced, float32, P(k, mu) with 5 mu bins
  and ell = 0, 2, 4: the whole FFTPower result against the float64 oracle,
  for the catalog in generator (cell) order and shuffled (the two routes of
  the bucketing).
* Zel'dovich lattice of 512^3 particles on a 1024^3 CIC interlaced float32
  mesh: too large for the oracle's full run inside a test, so it is checked
  on samples the oracle computes one by one (painted cells of both meshes,
  and the modes of the lowest k-bin summed directly over the particles), on
  the exact mode counts and mean |k| of all 512 bins, and on properties
  that hold at any size (mass conservation, Parseval of the r2c, finite
  results of the fused path).
* The largest mesh, 2048^3 CIC interlaced float32 (96 GiB of workspace): the
  fused path's lowest k-bins, P_0 and P_2 over 1 <= |n|^2 < 9, against the
  float64 oracle's modes computed one by one by direct summation over the
  particles (no mesh), with interlacing and compensation applied per mode.
"""

import concurrent.futures
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, synth
from tests.test_gpu_parity import check_power, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _fftpower(ctx, m, b, pos):
    ws = torch.empty(_lib.workspace_bytes(m, b, len(pos)), dtype=torch.uint8, device="cuda:0")
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower(m, b, pos, None, len(pos), ws, res)
    out = ctx.pk_result_to_host(m, b, res)
    del ws
    return out


@pytest.mark.timeout(600)
def test_lognormal_512_tsc_interlaced_full(ctx):
    n, box = 512, 1380.0
    pos = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 1e7 / n ** 3, seed=2)
    print(f"\nlognormal-512: {len(pos)} particles", flush=True)
    m = _lib.mesh_desc(n, box, "tsc", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 5, (0, 2, 4), 2)
    got = _fftpower(ctx, m, b, dev(pos))
    want = oracle.fftpower(pos.astype(np.float64), n, box, "tsc", True, True, nmu=5,
                           poles=(0, 2, 4))
    ok = want["modes"] > 0
    rel = np.abs(got["power"][ok] / want["power"][ok] - 1)
    print(f"max |dP/P| = {rel.max():.2e}", flush=True)
    check_power(got, want, 1e-5, "lognormal-512")
    # the same catalog in random order takes the other bucketing route
    # (slab partition instead of column runs) and must give the same result
    shuffled = pos[np.random.default_rng(12345).permutation(len(pos))]
    got_s = _fftpower(ctx, m, b, dev(shuffled))
    check_power(got_s, want, 1e-5, "lognormal-512 shuffled")
    np.testing.assert_allclose(got_s["power"][ok], got["power"][ok], rtol=1e-6)
    for ell in (0, 2, 4):
        np.testing.assert_allclose(got_s["poles"][ell][ok], got["poles"][ell][ok],
                                   rtol=0, atol=1e-6 * np.abs(got["power"][ok]).max())


def _plane_cells(rng, n, x0, count):
    cells = np.empty((count, 3), dtype=np.int64)
    cells[:, 0] = x0
    cells[:, 1:] = rng.integers(0, n, (count, 2))
    return cells


@pytest.mark.timeout(900)
def test_zeldovich_1024_cic_interlaced_sampled(ctx):
    n, box, ngrid = 1024, 2000.0, 512
    pos = synth.zeldovich_lattice(ngrid, box, synth.pk_zeldovich_c3, seed=3)
    print(f"\nzeldovich-1024: {len(pos)} particles", flush=True)
    pos_d = dev(pos)
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    got = _fftpower(ctx, m, b, pos_d)
    assert np.all(np.isfinite(got["power"][1:])) and np.all(np.isfinite(got["poles"][2][1:]))
    assert got["shotnoise"] == pytest.approx(box ** 3 / len(pos), rel=1e-12)
    tab = oracle.mode_tables(n, box, 0.0, 1.0, n // 2, interlaced=True)
    np.testing.assert_array_equal(got["modes"], tab["modes"])
    np.testing.assert_allclose(got["k"][1:], tab["k"][1:], rtol=1e-12)
    print("counts ok", flush=True)
    _check_low_k(got, pos, n, box, 2, kbins=(1,))

    rng = np.random.default_rng(0)
    u = oracle.cell_coordinates(pos.astype(np.float64), n, box)
    mesh = torch.empty((n, n, n), dtype=torch.float32, device="cuda:0")
    for shift in (0.0, 0.5):
        ctx.pk_paint(m, pos_d, None, len(pos), shift, mesh, None)
        total = float(mesh.sum(dtype=torch.float64))
        assert abs(total / len(pos) - 1) < 1e-6, total
        for x0 in (0, 517):
            # only particles within one cell of the plane can reach it (CIC)
            dx = u[:, 0] + shift - x0
            dx -= n * np.round(dx / n)
            near = np.abs(dx) < 1.0
            cells = _plane_cells(rng, n, x0, 48)
            want = oracle.paint_cells(pos[near].astype(np.float64), cells, n, box, 2,
                                      shift_cells=shift)
            idx = torch.from_numpy(cells).to("cuda:0")
            gotc = mesh[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
            np.testing.assert_allclose(gotc, want, rtol=0, atol=2e-6 * max(1.0, want.max()))
        print(f"sampled cells ok (shift {shift})", flush=True)

    # Parseval of the r2c on the painted mesh A: sum_modes h |c|^2 = N^3 sum F^2
    ctx.pk_paint(m, pos_d, None, len(pos), 0.0, mesh, None)
    f2 = float((mesh.double() ** 2).sum())
    ctx.pk_fft_r2c(m, mesh)
    c = mesh.view(n, n, n // 2, 2).double()
    p = c[..., 0] ** 2 + c[..., 1] ** 2
    lhs = float(p[:, :, 0].sum()) + 2.0 * float(p[:, :, 1:].sum())
    assert abs(lhs / (n ** 3 * f2) - 1) < 1e-5, lhs / (n ** 3 * f2)


@pytest.mark.timeout(900)
def test_max_mesh_2048_cic_interlaced_low_k_bins(ctx):
    n, box, ngrid = 2048, 2000.0, 192
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(16, 0.0, 1.0, 0, (0, 2), 2)
    pos = synth.zeldovich_lattice(ngrid, box, synth.pk_zeldovich_c3, seed=7)
    need = _lib.workspace_bytes(m, b, len(pos))
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    print(f"\n2048^3: {len(pos)} particles, workspace {need / 2**30:.1f} GiB", flush=True)
    got = _fftpower(ctx, m, b, dev(pos))
    torch.cuda.empty_cache()
    _check_low_k(got, pos, n, box, 2, kbins=(1, 2))


def _check_low_k(got, pos, n, box, order, kbins):
    """P_0 and P_2 of the lowest whole-number k-bins (unit weights, interlaced,
    compensated, line of sight z) against the oracle's modes summed directly
    over the particles, in chunks.  Half of the grid is summed (the other half
    are the complex conjugates, of equal power) and every mode counted twice."""
    top = max(kbins) + 1
    r = np.arange(-top, top + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    n2 = (g ** 2).sum(axis=1)
    half = (g[:, 2] > 0) | ((g[:, 2] == 0) & (g[:, 1] > 0)) | \
        ((g[:, 2] == 0) & (g[:, 1] == 0) & (g[:, 0] > 0))
    modes = g[(n2 >= min(kbins) ** 2) & (n2 < top ** 2) & half]
    # chunks of 4M particles on a thread pool (NumPy releases the GIL), the
    # partial sums added in chunk order
    def part(i0, shift):
        p64 = pos[i0:i0 + (1 << 22)].astype(np.float64)
        return oracle.painted_modes(p64, modes, n, box, order, None, shift)

    starts = range(0, len(pos), 1 << 22)
    with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        fa = [ex.submit(part, i0, 0.0) for i0 in starts]
        fb = [ex.submit(part, i0, 0.5) for i0 in starts]
        ca = sum(f.result() for f in fa)
        cb = sum(f.result() for f in fb)
    c = 0.5 * (ca + np.exp(1j * np.pi * modes.sum(axis=1) / n) * cb)
    c /= np.prod(np.sinc(modes / n), axis=1) ** order
    pw = box ** 3 * np.abs(c) ** 2 / float(len(pos)) ** 2
    n2m = (modes ** 2).sum(axis=1)
    mu2 = modes[:, 2] ** 2 / n2m
    kb = np.floor(np.sqrt(n2m)).astype(int)
    for k in kbins:
        sel = kb == k
        assert got["modes"][k] == 2 * sel.sum()
        p0 = pw[sel].mean()
        p2 = 5.0 * (pw[sel] * 0.5 * (3 * mu2[sel] - 1)).mean()
        print(f"bin {k}: P0 {got['power'][k]:.6e} oracle {p0:.6e}; "
              f"P2 {got['poles'][2][k]:.6e} oracle {p2:.6e}", flush=True)
        assert abs(got["power"][k] / p0 - 1) < 1e-5
        assert abs(got["poles"][2][k] - p2) < 1e-5 * abs(p0)
