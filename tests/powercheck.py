"""Comparison of a libpk FFTPower result with the oracle's, to the bar of
the float32 path: per bin |dP| / |P| <= tol for P(k) and P(k, mu),
|dP_ell| <= tol |P_0| for ell > 0 (P_ell can cross zero); mode counts bit
for bit; mean k and mu to float64 rounding."""

import numpy as np
import pytest


def check_power(got, want, tol, tag=""):
    np.testing.assert_array_equal(got["modes"], want["modes"], err_msg=f"{tag} counts")
    ok = want["modes"] > 0
    assert np.all(np.isnan(got["power"][~ok])), tag
    rel = np.abs(got["power"][ok] / want["power"][ok] - 1)
    assert rel.max() <= tol, f"{tag} P rel err {rel.max():.3e}"
    np.testing.assert_allclose(got["k"][ok], want["k"][ok], rtol=1e-13, err_msg=tag)
    for ell, p in want["poles"].items():
        err = np.abs(got["poles"][ell][ok] - p[ok]) / np.abs(want["power"][ok])
        assert err.max() <= tol, f"{tag} P_{ell} err {err.max():.3e}"
    if "modes2d" in want:
        np.testing.assert_array_equal(got["modes2d"], want["modes2d"], err_msg=f"{tag} 2d counts")
        ok2 = want["modes2d"] > 0
        rel2 = np.abs(got["power2d"][ok2] / want["power2d"][ok2] - 1)
        assert rel2.max() <= tol, f"{tag} P(k,mu) rel err {rel2.max():.3e}"
        np.testing.assert_allclose(got["mu2d"][ok2], want["mu2d"][ok2], rtol=1e-12, err_msg=tag)
        np.testing.assert_allclose(got["k2d"][ok2], want["k2d"][ok2], rtol=1e-12, err_msg=tag)
    assert got["shotnoise"] == pytest.approx(want["shotnoise"], rel=1e-12)
