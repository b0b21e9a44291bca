"""Comparison of a libpk FFTPower result with the oracle's, to the bar of
the float32 path: per bin |dP| / |P| <= tol for P(k) and P(k, mu),
|dP_ell| <= tol |P_0| for ell > 0 (P_ell can cross zero); mode counts bit
for bit.  The mean k and mu of a bin are float64 sums over up to ~10^7
modes taken in a different order on each side, so they get the float64
bar of the method, 1e-12 relative (the worst-case rounding of an n-term
float64 sum is ~n 2^-53, its typical size sqrt(n) 2^-53 ~ 1e-13 at
10^5 modes)."""

KBAR_RTOL = 1e-12

import numpy as np
import pytest


def check_power(got, want, tol, tag=""):
    np.testing.assert_array_equal(got["modes"], want["modes"], err_msg=f"{tag} counts")
    ok = want["modes"] > 0
    assert np.all(np.isnan(got["power"][~ok])), tag
    rel = np.abs(got["power"][ok] / want["power"][ok] - 1)
    assert rel.max() <= tol, f"{tag} P rel err {rel.max():.3e}"
    np.testing.assert_allclose(got["k"][ok], want["k"][ok], rtol=KBAR_RTOL, err_msg=tag)
    for ell, p in want["poles"].items():
        err = np.abs(got["poles"][ell][ok] - p[ok]) / np.abs(want["power"][ok])
        assert err.max() <= tol, f"{tag} P_{ell} err {err.max():.3e}"
    if "modes2d" in want:
        np.testing.assert_array_equal(got["modes2d"], want["modes2d"], err_msg=f"{tag} 2d counts")
        ok2 = want["modes2d"] > 0
        rel2 = np.abs(got["power2d"][ok2] / want["power2d"][ok2] - 1)
        assert rel2.max() <= tol, f"{tag} P(k,mu) rel err {rel2.max():.3e}"
        np.testing.assert_allclose(got["mu2d"][ok2], want["mu2d"][ok2], rtol=KBAR_RTOL,
                                   err_msg=tag)
        np.testing.assert_allclose(got["k2d"][ok2], want["k2d"][ok2], rtol=KBAR_RTOL, err_msg=tag)
    assert got["shotnoise"] == pytest.approx(want["shotnoise"], rel=1e-12)
