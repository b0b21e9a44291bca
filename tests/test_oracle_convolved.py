"""Pins of the survey-multipole oracle (ConvolvedFFTPower).

The paper names the estimator but does not spell it out (parity with the
paper is unpinned); the oracle's definitions are pinned by:
* the addition theorem of its real spherical harmonics, sum_m Y_lm(a) Y_lm(b)
  = (2 ell + 1) / (4 pi) L_ell(a . b), and their orthonormality by quadrature;
* a brute-force F_ell on a tiny mesh: every particle painted alone, weighted
  by L_ell(k^ . r^_i) mode by mode;
* the distant-observer limit, where the multipoles become the FFTPower
  multipoles of the same field along z.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import convolved as cv
from paper_1712_05834_amd import synth


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


@pytest.mark.parametrize("ell", [0, 2, 4])
def test_real_harmonics_addition_theorem(ell):
    rng = np.random.default_rng(ell + 1)
    a, b = _unit(rng, 200), _unit(rng, 200)
    lhs = sum(cv.real_ylm(ell, m, *a.T) * cv.real_ylm(ell, m, *b.T) for m in range(-ell, ell + 1))
    mu = np.sum(a * b, axis=1)
    rhs = (2 * ell + 1) / (4 * math.pi) * oracle.legendre(ell, mu * mu) if ell else \
        np.full(200, 1 / (4 * math.pi))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-14)


def test_real_harmonics_orthonormal():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for degree <= 8
    x, w = np.polynomial.legendre.leggauss(10)
    phi = 2 * math.pi * np.arange(20) / 20
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    wt = np.outer(w, np.full(20, 2 * math.pi / 20)).ravel()
    st = np.sqrt(1 - ct * ct)
    ux, uy, uz = (st * np.cos(ph)).ravel(), (st * np.sin(ph)).ravel(), ct.ravel()
    ylms = [(l, m, cv.real_ylm(l, m, ux, uy, uz)) for l in (0, 2, 4) for m in range(-l, l + 1)]
    for l1, m1, y1 in ylms:
        for l2, m2, y2 in ylms:
            g = np.sum(wt * y1 * y2)
            assert g == pytest.approx(1.0 if (l1, m1) == (l2, m2) else 0.0, abs=1e-12)


@pytest.mark.parametrize("ell", [0, 2, 4])
def test_multipole_field_brute_force(ell):
    n, box = 8, 10.0
    rng = np.random.default_rng(7 + ell)
    data = rng.uniform(0, box, (5, 3))
    rand = rng.uniform(0, box, (7, 3))
    wd, wr = rng.uniform(0.5, 1.5, 5), rng.uniform(0.5, 1.5, 7)
    obs = np.array([-3.0, 4.0, -20.0])
    fields, alpha, _ = cv.multipole_fields(data, rand, wd, wr, obs, n, box, "tsc", (ell,),
                                           compensated=False)
    khat = cv.k_unit_vectors(n)
    want = np.zeros_like(fields[ell])
    for pos, w, s in [(data, wd, 1.0), (rand, wr, -alpha)]:
        u = cv.unit_vectors(pos, obs)
        for i in range(len(pos)):
            one = oracle.r2c(oracle.paint_mesh(pos[i:i + 1], n, box, 3, np.array([s * w[i]])))
            mu = khat[0] * u[i, 0] + khat[1] * u[i, 1] + khat[2] * u[i, 2]
            lw = oracle.legendre(ell, mu * mu) if ell else np.ones_like(mu)
            want += lw * one
    sel = np.ones(want.shape, bool)
    sel[0, 0, 0] = False  # k^ undefined at DC
    np.testing.assert_allclose(fields[ell][sel], want[sel], rtol=1e-11, atol=1e-12)


def test_distant_observer_gives_fftpower_multipoles():
    n, box = 32, 500.0
    data = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 0.5, seed=3,
                                   dtype=np.float64)
    rand = synth.uniform_catalog(4 * len(data), box, seed=4)
    obs = np.array([box / 2, box / 2, -1e7 * box])
    norm = 2.5e-3
    got = cv.convolved_power(data, rand, None, None, obs, n, box, norm, "tsc", (0, 2, 4))
    alpha = len(data) / len(rand)
    field = oracle.paint_mesh(data, n, box, 3) - oracle.paint_mesh(rand, n, box, 3,
                                                                     np.full(len(rand), alpha))
    # FFTPower normalisation V / wsum^2 set equal to 1 / I
    want = oracle.fftpower_from_spectra(oracle.r2c(field), None, n, box, 3, True,
                                        math.sqrt(box ** 3 * norm), 0.0, 1, nmu=0,
                                        poles=(0, 2, 4))
    ok = want["modes"] > 0
    np.testing.assert_array_equal(got["modes"], want["modes"])
    scale = np.abs(want["poles"][0][ok])
    for ell in (0, 2, 4):
        err = np.abs(got["poles"][ell][ok] - want["poles"][ell][ok]) / scale
        assert err.max() < 1e-5, (ell, err.max())
    assert got["shotnoise"] == pytest.approx((len(data) + alpha ** 2 * len(rand)) / norm)


def test_periodic_images_give_the_same_multipoles():
    # the painting and the line of sight both take positions in the periodic
    # box: shifting particles by whole box lengths changes nothing
    n, box = 16, 100.0
    rng = np.random.default_rng(5)
    data, rand = rng.uniform(0, box, (300, 3)), rng.uniform(0, box, (900, 3))
    obs = np.array([50.0, 40.0, -80.0])
    a = cv.convolved_power(data, rand, None, None, obs, n, box, 1.0, "cic", (0, 2, 4))
    shift = rng.integers(-2, 3, (300, 3)) * box
    b = cv.convolved_power(data + shift, rand - box, None, None, obs, n, box, 1.0, "cic",
                           (0, 2, 4))
    for ell in (0, 2, 4):
        np.testing.assert_allclose(b["poles"][ell], a["poles"][ell], rtol=1e-9, atol=1e-9)
