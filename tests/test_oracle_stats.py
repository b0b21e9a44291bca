"""Statistical pins for the oracle estimator (Sec. 3.3 painting and Sec. 3.4.1).

* Shot noise: for N_p uniform random particles the expectation of the
  compensated per-mode power is exactly
      E[P(k)] = (V / N_p) prod_d S_p(theta_d) / prod_d sinc^{2p}(theta_d / 2)
  (interlaced: the mean of the plain and half-integer alias sums), which
  tends to V / N_p as k -> 0.  Checked as a z-score over independent modes.
* Gaussian fields: E[P_b] equals the mode average of the input P(k); the
  relative scatter of one bin is sqrt(2 / N_b).
"""

import numpy as np
import pytest

import oracle
from paper_1712_05834_amd import synth
from tests.test_oracle_spectral import s_half, s_int


def _theta(n):
    nx, ny, nz = oracle.mode_indices(n)
    return (2 * np.pi * nx / n)[:, None, None], (2 * np.pi * ny / n)[None, :, None], \
        (2 * np.pi * nz / n)[None, None, :]


def _sinc(x):
    return np.sinc(x / np.pi)


@pytest.mark.parametrize("order,interlaced", [(2, False), (3, False), (4, False),
                                              (2, True), (3, True)])
def test_shot_noise_expectation(order, interlaced):
    n, box, npart = 32, 1000.0, 40000
    pos = synth.uniform_catalog(npart, box, seed=100 + order)
    ca = oracle.r2c(oracle.paint_mesh(pos, n, box, order))
    if interlaced:
        cb = oracle.r2c(oracle.paint_mesh(pos, n, box, order, shift_cells=0.5))
        ca = oracle.interlace_combine(ca, cb, n)
    c = oracle.compensate(ca, n, order)
    pmode = box ** 3 * np.abs(c) ** 2 / npart ** 2
    tx, ty, tz = _theta(n)
    alias = s_int(order, tx) * s_int(order, ty) * s_int(order, tz)
    if interlaced:
        alias = 0.5 * (alias + s_half(order, tx) * s_half(order, ty) * s_half(order, tz))
    window = (_sinc(tx / 2) * _sinc(ty / 2) * _sinc(tz / 2)) ** (2 * order)
    expect = box ** 3 / npart * alias / window
    # independent modes: 0 < n_z < N/2 (each mode appears once)
    ratio = (pmode / expect)[:, :, 1 : n // 2]
    z = np.sum(ratio - 1.0) / np.sqrt(ratio.size)
    assert abs(z) < 5.0, z
    # the low-k limit is V / N_p
    assert abs(expect[1, 0, 0] * npart / box ** 3 - 1) < 1e-3
    # and through the full estimator: bin means against binned expectations
    res = oracle.fftpower(pos, n, box, window=order, interlaced=interlaced)
    assert res["shotnoise"] == pytest.approx(box ** 3 / npart, rel=1e-14)
    h = np.ones(n // 2 + 1)
    h[1 : n // 2] = 2
    n2 = (np.fft.fftfreq(n, 1 / n)[:, None, None] ** 2 + np.fft.fftfreq(n, 1 / n)[None, :, None] ** 2
          + np.arange(n // 2 + 1)[None, None, :] ** 2)
    b = np.floor(np.sqrt(n2)).astype(int)
    eb = np.zeros(n // 2)
    for k in range(1, n // 2):
        m = (b == k) & (n2 > 0)
        eb[k] = np.sum((h * expect)[m]) / np.sum((h + 0 * expect)[m])
    sel = res["modes"] > 0
    zb = (res["power"][sel] / eb[sel] - 1) / np.sqrt(2.0 / res["modes"][sel])
    assert np.all(np.abs(zb) < 5.5), zb


def test_gaussian_field_recovers_input_power():
    n, box, nseed = 32, 800.0, 8
    pk = synth.pk_lognormal_c2
    acc = None
    for s in range(nseed):
        delta = synth.gaussian_field(n, box, pk, seed=300 + s)
        res = oracle.fftpower_from_spectra(oracle.r2c(1.0 + delta), None, n, box, 2, False,
                                           float(n ** 3), 1.0, 1)
        acc = res["power"] if acc is None else acc + res["power"]
    mean = acc / nseed
    # expected: mode average of P(|k|) (full-grid enumeration)
    r = np.arange(-n // 2, n // 2)
    g = np.meshgrid(r, r, r, indexing="ij")
    n2 = (g[0] ** 2 + g[1] ** 2 + g[2] ** 2).ravel()
    b = np.floor(np.sqrt(n2)).astype(int)
    kf = 2 * np.pi / box
    sel = (n2 > 0) & (b < n // 2)
    want = np.bincount(b[sel], weights=pk(kf * np.sqrt(n2[sel])), minlength=n // 2) / \
        np.bincount(b[sel], minlength=n // 2)
    ok = res["modes"] > 0
    z = (mean[ok] / want[ok] - 1) / np.sqrt(2.0 / (nseed * res["modes"][ok]))
    assert np.all(np.abs(z) < 5), z
    chi2 = np.mean(z ** 2)
    assert 0.3 < chi2 < 2.5, chi2


def test_weighted_paint_normalisation_and_shot_noise():
    n, box, npart = 16, 300.0, 5000
    pos = synth.uniform_catalog(npart, box, seed=7)
    w = synth.uniform_weights(npart, seed=8)
    res = oracle.fftpower(pos, n, box, window="tsc", weight=w)
    assert res["wsum"] == pytest.approx(w.sum(), rel=1e-14)
    assert res["w2sum"] == pytest.approx((w * w).sum(), rel=1e-14)
    assert res["shotnoise"] == pytest.approx(box ** 3 * (w * w).sum() / w.sum() ** 2, rel=1e-14)
    # doubling every weight leaves the normalised power unchanged
    res2 = oracle.fftpower(pos, n, box, window="tsc", weight=2 * w)
    np.testing.assert_allclose(res2["power"], res["power"], rtol=1e-13, equal_nan=True)
