"""Pins of the oracle's variants: value painting and the cross power.

* Cross power: for a field and a copy of it shifted by s cells along an axis,
  the modes differ by the phase exp(-2 pi i n_a s / N), so the cross power of
  a fixed-amplitude field is exactly the mode average of P(|k|) cos(2 pi n_a
  s / N), checked by brute-force enumeration of the full grid; the cross power
  of a field with itself is its auto power; Cauchy-Schwarz bounds every bin.
* Value painting (Sec. 3.3.1, F = [1 + delta'] V): a constant value c scales
  P and the shot noise by c^2 (the normalisation stays sum w); painting w V
  equals painting with weights w V renormalised by (sum w V / sum w)^2.
"""

import math

import numpy as np
import pytest

import oracle
from paper_1712_05834_amd import synth


def _full_grid(n):
    r = np.arange(-n // 2, n // 2)
    g = np.meshgrid(r, r, r, indexing="ij")
    return g[0].ravel(), g[1].ravel(), g[2].ravel()


@pytest.mark.parametrize("axis,shift", [(0, 1), (2, 3), (1, 5)])
def test_cross_of_shifted_fixed_amplitude_field_is_exact(axis, shift):
    n, box, nk = 16, 300.0, 8
    pk = synth.pk_lognormal_c2
    f1 = synth.fixed_amplitude_field(n, box, pk, seed=31)
    f2 = np.roll(f1, shift, axis=axis)
    c1, c2 = oracle.r2c(f1), oracle.r2c(f2)
    w = float(n ** 3)
    res = oracle.cross_from_spectra(c1, c2, n, box, w, w, nk=nk)
    # brute force: mode average of P(|k|) cos(2 pi n_a s / N) over the full grid
    gx, gy, gz = _full_grid(n)
    n2 = gx * gx + gy * gy + gz * gz
    b = np.array([math.isqrt(int(v)) for v in n2])
    sel = (n2 > 0) & (b < nk)
    kf = 2 * np.pi / box
    na = (gx, gy, gz)[axis][sel]
    p = pk(kf * np.sqrt(n2[sel].astype(np.float64))) * np.cos(2 * np.pi * na * shift / n)
    cnt = np.bincount(b[sel], minlength=nk)
    want = np.bincount(b[sel], weights=p, minlength=nk) / np.where(cnt > 0, cnt, 1)
    ok = cnt > 0
    np.testing.assert_array_equal(res["modes"], cnt)
    np.testing.assert_allclose(res["power"][ok], want[ok], rtol=0,
                               atol=1e-12 * np.abs(want[ok]).max())
    # symmetric in its two fields
    res21 = oracle.cross_from_spectra(c2, c1, n, box, w, w, nk=nk)
    np.testing.assert_array_equal(res21["power"], res["power"])


def test_cross_with_itself_is_the_auto_power():
    n, box = 32, 400.0
    pos = synth.uniform_catalog(3000, box, seed=41)
    wts = synth.uniform_weights(3000, seed=42)
    c, wsum = oracle.prepared_spectrum(pos, n, box, "tsc", True, True, wts)
    cross = oracle.cross_from_spectra(c, c, n, box, wsum, wsum, nmu=3, poles=(0, 2),
                                      interlaced=True)
    auto = oracle.fftpower(pos, n, box, "tsc", True, True, wts, nmu=3, poles=(0, 2))
    ok = auto["modes"] > 0
    np.testing.assert_allclose(cross["power"][ok], auto["power"][ok], rtol=1e-13)
    np.testing.assert_allclose(cross["poles"][2][ok], auto["poles"][2][ok], rtol=1e-12,
                               atol=1e-13 * np.abs(auto["power"][ok]).max())
    ok2 = auto["modes2d"] > 0
    np.testing.assert_allclose(cross["power2d"][ok2], auto["power2d"][ok2], rtol=1e-13)
    assert cross["shotnoise"] == 0.0


def test_cross_power_obeys_cauchy_schwarz():
    n, box = 16, 200.0
    c1, w1 = oracle.prepared_spectrum(synth.uniform_catalog(500, box, seed=51), n, box, "cic")
    c2, w2 = oracle.prepared_spectrum(synth.uniform_catalog(700, box, seed=52), n, box, "cic")
    x = oracle.cross_from_spectra(c1, c2, n, box, w1, w2)
    a1 = oracle.cross_from_spectra(c1, c1, n, box, w1, w1)
    a2 = oracle.cross_from_spectra(c2, c2, n, box, w2, w2)
    ok = x["modes"] > 0
    assert np.all(np.abs(x["power"][ok]) <= np.sqrt(a1["power"][ok] * a2["power"][ok]) * (1 + 1e-12))
    # independent catalogs: the cross power is far below the auto powers
    assert np.mean(np.abs(x["power"][ok])) < 0.5 * np.mean(np.sqrt(a1["power"][ok] * a2["power"][ok]))


def test_constant_value_scales_power_by_its_square():
    n, box = 32, 500.0
    pos = synth.uniform_catalog(4000, box, seed=61)
    base = oracle.fftpower(pos, n, box, "cic", True, nmu=2, poles=(0, 2))
    one = oracle.fftpower(pos, n, box, "cic", True, nmu=2, poles=(0, 2), value=np.ones(4000))
    val = oracle.fftpower(pos, n, box, "cic", True, nmu=2, poles=(0, 2),
                          value=np.full(4000, 2.5))
    ok = base["modes"] > 0
    np.testing.assert_array_equal(one["power"][ok], base["power"][ok])
    np.testing.assert_allclose(val["power"][ok], 6.25 * base["power"][ok], rtol=1e-12)
    np.testing.assert_allclose(val["poles"][2][ok], 6.25 * base["poles"][2][ok], rtol=1e-11,
                               atol=1e-12 * base["power"][ok].max())
    assert val["shotnoise"] == pytest.approx(6.25 * base["shotnoise"], rel=1e-12)


def test_value_painting_normalises_by_the_weights_alone():
    n, box, npart = 32, 500.0, 3000
    pos = synth.uniform_catalog(npart, box, seed=71)
    w = synth.uniform_weights(npart, seed=72)
    v = synth.rng_for(73).normal(0.0, 300.0, npart)  # e.g. a velocity component
    val = oracle.fftpower(pos, n, box, "tsc", False, True, w, value=v)
    asw = oracle.fftpower(pos, n, box, "tsc", False, True, w * v)
    ratio = (np.sum(w * v) / np.sum(w)) ** 2
    ok = val["modes"] > 0
    np.testing.assert_allclose(val["power"][ok], ratio * asw["power"][ok], rtol=1e-10)
    assert val["wsum"] == pytest.approx(np.sum(w), rel=1e-15)
    assert val["shotnoise"] == pytest.approx(box ** 3 * np.sum((w * v) ** 2) / np.sum(w) ** 2,
                                             rel=1e-12)
    # the painted mesh conserves sum w V
    mesh = oracle.paint_mesh(pos, n, box, 3, w * v)
    assert mesh.sum() == pytest.approx(np.sum(w * v), rel=1e-10)


@pytest.mark.parametrize("keep", [(0, 1), (2,), (1, 2), (0,)])
def test_projected_power_is_the_zero_plane_of_the_3d_spectrum(keep):
    """The d-dimensional DFT of the field summed over the projected axes equals
    the 3-D DFT on the plane where the projected wave numbers vanish; the
    projected power built from the 3-D spectrum that way matches."""
    n, box, nk = 16, 200.0, 8
    pos = synth.uniform_catalog(800, box, seed=81)
    res = oracle.projected_power(pos, n, box, keep, "tsc", interlaced=True, nk=nk)
    # independent route: full 3-D transform of both meshes, interlace and
    # compensate in 3-D, then keep the modes with n = 0 on the projected axes
    c3a = np.fft.fftn(oracle.paint_mesh(pos, n, box, 3))
    c3b = np.fft.fftn(oracle.paint_mesh(pos, n, box, 3, None, 0.5))
    f = np.arange(n)
    f = np.where(f < n // 2, f, f - n)
    gx, gy, gz = np.meshgrid(f, f, f, indexing="ij")
    c3 = 0.5 * (c3a + np.exp(1j * np.pi * (gx + gy + gz) / n) * c3b)
    for g in (gx, gy, gz):
        c3 = c3 / np.sinc(g / n) ** 3  # numpy sinc(x) = sin(pi x) / (pi x)
    drop = [a for a in range(3) if a not in keep]
    sel = np.ones(c3.shape, bool)
    for a in drop:
        sel &= (gx, gy, gz)[a] == 0
    n2 = (gx * gx + gy * gy + gz * gz)[sel]
    p = box ** len(keep) * np.abs(c3[sel]) ** 2 / 800.0 ** 2
    b = np.array([math.isqrt(int(v)) for v in n2])
    ok = (n2 > 0) & (b < nk)
    cnt = np.bincount(b[ok], minlength=nk)
    want = np.bincount(b[ok], weights=p[ok], minlength=nk) / np.where(cnt > 0, cnt, 1)
    np.testing.assert_array_equal(res["modes"], cnt)
    good = cnt > 0
    np.testing.assert_allclose(res["power"][good], want[good], rtol=1e-10)
    assert res["shotnoise"] == pytest.approx(box ** len(keep) / 800.0, rel=1e-12)


def test_projected_power_of_uniform_catalog_is_shot_noise():
    """For a Poisson catalog the projected power averages to L^d / N (times the
    window alias sums, close to 1 at low k once compensated)."""
    n, box, npart = 64, 1000.0, 200000
    pos = synth.uniform_catalog(npart, box, seed=91)
    res = oracle.projected_power(pos, n, box, (0, 1), "cic", interlaced=True, nk=8)
    ok = res["modes"] > 0
    ratio = res["power"][ok] / res["shotnoise"]
    # low-k bins: |ratio - 1| within 4 sigma of the chi^2 scatter sqrt(1 / N_b)
    assert np.all(np.abs(ratio - 1) < 4 / np.sqrt(res["modes"][ok]) + 0.02)
