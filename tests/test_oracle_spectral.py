"""Pins for the oracle's r2c transform, interlacing and compensation.

Sec. 3.3.1 (r2c), Sec. 3.3.2 (interlacing; Eq. 2 compensation).

Expected values come from mathematics only:
* a brute-force O(N^6) DFT, a single plane wave and Parseval's identity;
* the exact alias sums of a single particle averaged over its sub-cell offset:
  E|c(k)|^2 = prod_d S_p(theta_d) with S_p(theta) = sum_j M_2p(j) e^{-i theta j},
  and for the interlaced pair (1/2)[prod S_p + prod S'_p] with
  S'_p(theta) = sum_j M_2p(j + 1/2) e^{-i theta (j + 1/2)};  M_2p are the
  order-2p B-spline values at integers / half-integers (exact rationals);
* E[c(k) e^{i k.x_p}] over the sub-cell offset equals the window's continuous
  transform prod sinc^p(theta_d / 2), so the compensated average is exactly 1;
* node particles: CIC c_int e^{i k.x_p} = (1 + prod cos(theta_d / 2)) / 2 and
  TSC (prod(3/4 + cos(theta_d) / 4) + prod cos(theta_d / 2)) / 2.
The averages over the sub-cell offset use Gauss-Legendre nodes on [0, 1/2] and
[1/2, 1]: the integrands are polynomials of degree 2(p - 1) on each piece, so
p + 1 nodes per piece integrate them exactly.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle

# order-2p B-spline values at integers j >= 0 and half-integers j + 1/2
M_INT = {
    2: [Fraction(2, 3), Fraction(1, 6)],
    3: [Fraction(11, 20), Fraction(13, 60), Fraction(1, 120)],
    4: [Fraction(151, 315), Fraction(397, 1680), Fraction(1, 42), Fraction(1, 5040)],
}
M_HALF = {
    2: [Fraction(23, 48), Fraction(1, 48)],
    3: [Fraction(841, 1920), Fraction(79, 1280), Fraction(1, 3840)],
    4: [Fraction(259723, 645120), Fraction(20219, 215040), Fraction(2179, 645120),
        Fraction(1, 645120)],
}


def s_int(order, theta):
    m = [float(v) for v in M_INT[order]]
    out = m[0] * np.ones_like(theta)
    for j in range(1, len(m)):
        out = out + 2.0 * m[j] * np.cos(j * theta)
    return out


def s_half(order, theta):
    m = [float(v) for v in M_HALF[order]]
    out = np.zeros_like(theta)
    for j in range(len(m)):
        out = out + 2.0 * m[j] * np.cos((j + 0.5) * theta)
    return out


def test_bspline_tables_are_normalised_and_match_convolution():
    # partition of unity at integers and half-integers (exact rationals)
    for order in (2, 3, 4):
        assert M_INT[order][0] + 2 * sum(M_INT[order][1:]) == 1
        assert 2 * sum(M_HALF[order]) == 1
    # and the values are those of the order-2p B-spline (numerical convolution)
    from tests.test_oracle_window import _box_convolution_bspline
    for order in (2, 3, 4):
        j = np.arange(len(M_INT[order]), dtype=np.float64)
        np.testing.assert_allclose(_box_convolution_bspline(2 * order, j),
                                   [float(v) for v in M_INT[order]], atol=5e-6)
        np.testing.assert_allclose(_box_convolution_bspline(2 * order, j + 0.5),
                                   [float(v) for v in M_HALF[order]], atol=5e-6)


def _theta(n):
    nx, ny, nz = oracle.mode_indices(n)
    return (2 * np.pi * nx / n)[:, None, None], (2 * np.pi * ny / n)[None, :, None], \
        (2 * np.pi * nz / n)[None, None, :]


def test_r2c_matches_brute_dft():
    n = 8
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n, n, n))
    idx = np.arange(n)
    e = np.exp(-2j * np.pi * np.outer(idx, idx) / n)  # e[k, x]
    want = np.einsum("ax,by,cz,xyz->abc", e, e, e[: n // 2 + 1], f)
    got = oracle.r2c(f)
    assert got.shape == (n, n, n // 2 + 1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_r2c_plane_wave_single_mode():
    n = 16
    x = np.arange(n)
    g = np.meshgrid(x, x, x, indexing="ij")
    f = np.cos(2 * np.pi * (3 * g[0] + 1 * g[1] + 2 * g[2]) / n)
    c = oracle.r2c(f)
    assert abs(c[3, 1, 2] - n ** 3 / 2) < 1e-9
    c[3, 1, 2] = 0
    assert np.abs(c).max() < 1e-9


def test_c2r_matches_brute_backward_sum_and_inverts_r2c():
    # the backward sum over the full grid, the half spectrum's other half
    # taken as the complex conjugate, written out by hand
    n = 8
    rng = np.random.default_rng(2)
    f = rng.standard_normal((n, n, n))
    c = oracle.r2c(f)
    full = np.empty((n, n, n), dtype=np.complex128)
    full[:, :, : n // 2 + 1] = c
    for kz in range(n // 2 + 1, n):
        full[:, :, kz] = np.conj(c[(-np.arange(n)) % n][:, (-np.arange(n)) % n, n - kz])
    idx = np.arange(n)
    e = np.exp(2j * np.pi * np.outer(idx, idx) / n)  # e[x, k]
    want = np.einsum("xa,yb,zc,abc->xyz", e, e, e, full)
    got = oracle.c2r(c, n)
    np.testing.assert_allclose(got, want.real, rtol=0, atol=1e-10 * np.abs(want).max())
    np.testing.assert_allclose(got, n ** 3 * f, rtol=0, atol=1e-9)


def test_parseval_half_grid_weights():
    n = 16
    f = np.random.default_rng(2).standard_normal((n, n, n))
    c = oracle.r2c(f)
    nz = np.arange(n // 2 + 1)
    h = np.where((nz == 0) | (nz == n // 2), 1.0, 2.0)
    lhs = np.sum(h[None, None, :] * np.abs(c) ** 2)
    assert abs(lhs - n ** 3 * np.sum(f * f)) < 1e-12 * lhs


def _gl_nodes(m):
    """Gauss-Legendre nodes and weights on [0, 1/2] and [1/2, 1], weights sum to 1."""
    x, w = np.polynomial.legendre.leggauss(m)
    t = np.concatenate([0.25 + 0.25 * x, 0.75 + 0.25 * x])
    wt = np.concatenate([0.25 * w, 0.25 * w])
    return t, wt


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("interlaced", [False, True])
def test_single_particle_alias_sum(order, interlaced):
    n, box = 8, 8.0  # H = 1, so u = x
    t, wt = _gl_nodes(order + 1)
    acc = np.zeros((n, n, n // 2 + 1))
    base = np.array([3.0, 2.0, 5.0])
    for a, wa in zip(t, wt):
        for b, wb in zip(t, wt):
            for c, wc in zip(t, wt):
                pos = (base + [a, b, c])[None, :]
                ca = oracle.r2c(oracle.paint_mesh(pos, n, box, order))
                if interlaced:
                    cb = oracle.r2c(oracle.paint_mesh(pos, n, box, order, shift_cells=0.5))
                    ca = oracle.interlace_combine(ca, cb, n)
                acc += wa * wb * wc * np.abs(ca) ** 2
    tx, ty, tz = _theta(n)
    want = s_int(order, tx) * s_int(order, ty) * s_int(order, tz)
    if interlaced:
        want = 0.5 * (want + s_half(order, tx) * s_half(order, ty) * s_half(order, tz))
    np.testing.assert_allclose(acc, want, rtol=0, atol=1e-13)


def test_interlace_phase_sign_is_discriminated():
    """With the opposite phase sign the interlaced alias sum is far off."""
    n, box, order = 8, 8.0, 2
    t, wt = _gl_nodes(order + 1)
    nx, ny, nz = oracle.mode_indices(n)
    s = nx[:, None, None] + ny[None, :, None] + nz[None, None, :]
    wrong = np.exp(-1j * np.pi * s / n)
    acc = np.zeros((n, n, n // 2 + 1))
    for a, wa in zip(t, wt):
        for b, wb in zip(t, wt):
            for c, wc in zip(t, wt):
                pos = (np.array([1.0, 6.0, 4.0]) + [a, b, c])[None, :]
                ca = oracle.r2c(oracle.paint_mesh(pos, n, box, order))
                cb = oracle.r2c(oracle.paint_mesh(pos, n, box, order, shift_cells=0.5))
                acc += wa * wb * wc * np.abs(0.5 * (ca + wrong * cb)) ** 2
    tx, ty, tz = _theta(n)
    want = 0.5 * (s_int(order, tx) * s_int(order, ty) * s_int(order, tz)
                  + s_half(order, tx) * s_half(order, ty) * s_half(order, tz))
    assert np.abs(acc - want).max() > 0.1


@pytest.mark.parametrize("order", [2, 3])
def test_node_particle_interlaced_closed_form(order):
    n, box = 16, 32.0
    u = np.array([5, 9, 2])
    pos = (u * box / n)[None, :]
    ca = oracle.r2c(oracle.paint_mesh(pos, n, box, order))
    cb = oracle.r2c(oracle.paint_mesh(pos, n, box, order, shift_cells=0.5))
    c = oracle.interlace_combine(ca, cb, n)
    tx, ty, tz = _theta(n)
    got = c * np.exp(1j * (tx * u[0] + ty * u[1] + tz * u[2]))
    half = np.cos(tx / 2) * np.cos(ty / 2) * np.cos(tz / 2)
    if order == 2:
        want = 0.5 * (1 + half)
    else:
        want = 0.5 * ((0.75 + 0.25 * np.cos(tx)) * (0.75 + 0.25 * np.cos(ty))
                      * (0.75 + 0.25 * np.cos(tz)) + half)
    np.testing.assert_allclose(got, want + 0j, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_compensation_inverts_window_transform(order, axis):
    """Averaged over the sub-cell offset, c(k) e^{i k x_p} = sinc^p(theta / 2),
    so the compensated average is exactly 1 on every mode along the axis."""
    n, box = 16, 16.0
    t, wt = _gl_nodes(16)
    acc = np.zeros(n if axis < 2 else n // 2 + 1, dtype=complex)
    base = np.array([4.0, 7.0, 11.0])
    th = 2 * np.pi * oracle.mode_indices(n)[axis] / n
    for a, wa in zip(t, wt):
        pos = base.copy()
        pos[axis] += a
        c = oracle.compensate(oracle.r2c(oracle.paint_mesh(pos[None, :], n, box, order)),
                              n, order)
        line = [c[:, 0, 0], c[0, :, 0], c[0, 0, :]][axis]
        acc += wa * line * np.exp(1j * th * pos[axis])
    np.testing.assert_allclose(acc, 1.0 + 0j, rtol=0, atol=1e-12)
