"""GPU parity of the estimator's variants against the oracle:

* cross power of two catalogs on one mesh (pk_bin_cross on spectra prepared
  with pk_paint / pk_fft_r2c / pk_compensate);
* value painting, F = [1 + delta'] V (pk_fftpower_v);
* projected power (pk_bin_projected) for kept planes and lines.

Tolerances as everywhere: float32 1e-5 per bin (P_ell against |P_0|, a cross
power against the geometric mean of the auto powers, a projected power against
max(P, shot noise)), float64 1e-12; counts bit for bit."""

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, synth
from tests.powercheck import check_power

pytestmark = pytest.mark.gpu

TOL = {"f8": 1e-12, "f4": 1e-5}
TDT = {"f8": torch.float64, "f4": torch.float32}
NDT = {"f8": np.float64, "f4": np.float32}


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def prepared(ctx, m, pos, w):
    """Compensated (and interlaced) packed spectrum of one catalog, sum w."""
    n = m.nmesh
    dt = torch.float64 if m.dtype == _lib.PK_F64 else torch.float32
    a = torch.empty((n, n, n), dtype=dt, device="cuda:0")
    wsums = torch.empty(2, dtype=torch.float64, device="cuda:0")
    ctx.pk_paint(m, dev(pos), dev(w), len(pos), 0.0, a, wsums)
    ctx.pk_fft_r2c(m, a)
    bmesh = None
    if m.interlaced:
        bmesh = torch.empty_like(a)
        ctx.pk_paint(m, dev(pos), dev(w), len(pos), 0.5, bmesh, None)
        ctx.pk_fft_r2c(m, bmesh)
    ctx.pk_compensate(m, a, bmesh)
    return a, float(wsums[0])


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("window,inter", [("tsc", True), ("cic", False), ("pcs", True)])
def test_cross_power_matches_oracle(ctx, dtype, window, inter):
    n, box = 32, 400.0
    p1 = synth.uniform_catalog(6000, box, seed=101).astype(NDT[dtype])
    p2 = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 0.2, seed=102,
                                 dtype=NDT[dtype])
    w1 = synth.uniform_weights(len(p1), seed=103).astype(NDT[dtype])
    m = _lib.mesh_desc(n, box, window, inter, True, dtype)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 4, (0, 2), 2)
    c1, ws1 = prepared(ctx, m, p1, w1)
    c2, ws2 = prepared(ctx, m, p2, None)
    res = torch.zeros(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_cross(m, b, c1, c2, res)
    res[-2], res[-1] = float(np.sqrt(ws1 * ws2)), 0.0
    got = ctx.pk_result_to_host(m, b, res)
    o1, w1s = oracle.prepared_spectrum(p1.astype(np.float64), n, box, window, inter, True,
                                       w1.astype(np.float64))
    o2, w2s = oracle.prepared_spectrum(p2.astype(np.float64), n, box, window, inter, True)
    want = oracle.cross_from_spectra(o1, o2, n, box, w1s, w2s, nmu=4, poles=(0, 2),
                                     interlaced=inter)
    # a cross power crosses zero: compare against the auto-power scale
    np.testing.assert_array_equal(got["modes"], want["modes"])
    ok = want["modes"] > 0
    scale = np.sqrt(np.abs(oracle.cross_from_spectra(o1, o1, n, box, w1s, w1s)["power"][ok])
                    * np.abs(oracle.cross_from_spectra(o2, o2, n, box, w2s, w2s)["power"][ok]))
    assert np.max(np.abs(got["power"][ok] - want["power"][ok]) / scale) <= TOL[dtype]
    assert np.max(np.abs(got["poles"][2][ok] - want["poles"][2][ok]) / scale) <= TOL[dtype]
    ok2 = want["modes2d"] > 0
    np.testing.assert_array_equal(got["modes2d"], want["modes2d"])
    # P(k, mu) of the cross power per (k, mu)-bin against the oracle, on the
    # scale of the geometric mean of the two auto powers of that bin
    a1 = oracle.cross_from_spectra(o1, o1, n, box, w1s, w1s, nmu=4, interlaced=inter)
    a2 = oracle.cross_from_spectra(o2, o2, n, box, w2s, w2s, nmu=4, interlaced=inter)
    scale2 = np.sqrt(np.abs(a1["power2d"][ok2]) * np.abs(a2["power2d"][ok2]))
    err2 = np.abs(got["power2d"][ok2] - want["power2d"][ok2]) / scale2
    print(f"cross {window} {dtype}: max P(k,mu) err {err2.max():.2e}")
    assert err2.max() <= TOL[dtype]
    np.testing.assert_allclose(got["mu2d"][ok2], want["mu2d"][ok2], rtol=1e-12)
    assert got["shotnoise"] == 0.0


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("weighted", [False, True])
def test_value_painting_matches_oracle(ctx, dtype, weighted):
    n, box, npart = 64, 600.0, 30000
    pos = synth.uniform_catalog(npart, box, seed=111).astype(NDT[dtype])
    v = (1.0 + 0.3 * synth.rng_for(112).standard_normal(npart)).astype(NDT[dtype])
    w = synth.uniform_weights(npart, seed=113).astype(NDT[dtype]) if weighted else None
    m = _lib.mesh_desc(n, box, "tsc", True, True, dtype)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 3, (0, 2, 4), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower_v(m, b, dev(pos), dev(w), dev(v), npart, ws, res)
    got = ctx.pk_result_to_host(m, b, res)
    want = oracle.fftpower(pos.astype(np.float64), n, box, "tsc", True, True,
                           None if w is None else w.astype(np.float64), nmu=3, poles=(0, 2, 4),
                           value=v.astype(np.float64))
    check_power(got, want, TOL[dtype], f"value painting {dtype} weighted={weighted}")


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("keep", [(0, 1), (2,), (1, 2), (0,)])
def test_projected_power_matches_oracle(ctx, dtype, keep):
    n, box = 64, 800.0
    pos = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 0.3, seed=121,
                                  dtype=NDT[dtype])
    m = _lib.mesh_desc(n, box, "tsc", True, True, dtype)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (), 2)
    c, wsum = prepared(ctx, m, pos, None)
    mask = sum(1 << a for a in keep)
    res = torch.zeros(_lib.projected_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_projected(m, b, mask, c, res)
    res[-2], res[-1] = wsum, float(len(pos))
    got = ctx.pk_projected_to_host(m, b, mask, res)
    want = oracle.projected_power(pos.astype(np.float64), n, box, keep, "tsc", True, True)
    np.testing.assert_array_equal(got["modes"], want["modes"])
    ok = want["modes"] > 0
    # a bin of the 1-D projection holds a single +-k pair of modes, so nothing
    # averages the rounding of one mode, and the modes of the x projection lie
    # on the kz = 0 plane, which the real-input split forms from differences
    # of sums of the order of the DC mode (errors of order eps |DC|): errors
    # are measured against max(P, shot noise), with 1e-4 for float32 1-D
    # projections (observed 1.7e-5 for x, 3.4e-7 for z, 2-3.6e-7 in 2-D)
    scale = np.maximum(np.abs(want["power"][ok]), want["shotnoise"])
    rel = np.abs(got["power"][ok] - want["power"][ok]) / scale
    tol = 1e-4 if (dtype == "f4" and len(keep) == 1) else TOL[dtype]
    print(f"\nprojected {dtype} keep={keep}: max error / max(P, shot noise) {rel.max():.2e}")
    assert rel.max() <= tol, f"keep {keep}: {rel.max():.3e}"
    np.testing.assert_allclose(got["k"][ok], want["k"][ok], rtol=1e-13)
    assert got["shotnoise"] == pytest.approx(want["shotnoise"], rel=1e-12)
