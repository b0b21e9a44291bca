"""Pins for the oracle's painting (Sec. 3.3.1 Eq. 1, Sec. 3.3.2 windows).

Every expected value here comes from mathematics, not from the oracle:
B-splines built by numerically convolving unit boxes, exact rational window
values, brute-force per-cell sums over periodic images, and exact invariants
(partition of unity, mass conservation, whole-cell shifts).
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.paint import bspline


def _box_convolution_bspline(order, a, h=1.0 / 2000):
    """M_p(a) as the p-fold convolution of the unit box, built numerically.

    The exact tent M_2 on a grid of spacing h is convolved p - 2 more times
    with the unit box (trapezoid weights), then linearly interpolated at a.
    Independent of the oracle's closed-form piecewise polynomials; accurate
    to O(h^2).
    """
    k = int(round(0.5 / h))
    box = np.ones(2 * k + 1)
    box[0] = box[-1] = 0.5
    x = np.arange(-int(round(1.0 / h)), int(round(1.0 / h)) + 1) * h
    m = np.maximum(0.0, 1.0 - np.abs(x))
    for _ in range(order - 2):
        m = np.convolve(m, box) * h
        x = np.arange(len(m)) * h - (len(m) // 2) * h
    return np.interp(a, x, m, left=0.0, right=0.0)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_bspline_matches_box_convolution(order):
    a = np.linspace(-2.3, 2.3, 47)
    want = _box_convolution_bspline(order, a)
    np.testing.assert_allclose(bspline(order, a), want, atol=2e-6)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_partition_of_unity(order):
    rng = np.random.default_rng(11)
    u = rng.uniform(0, 64, 2000)
    cells, w = oracle.window_weights(u, order)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=2e-15)
    # the window is centred: first moment sum_j w_j j equals u
    np.testing.assert_allclose((w * cells).sum(axis=1), u, rtol=0, atol=1e-12)
    assert np.all(w >= 0)


def test_exact_rational_window_values():
    cases = [
        # (order, u, first cell, exact weights)
        (2, 3.25, 3, [Fraction(3, 4), Fraction(1, 4)]),
        (3, 5.125, 4, [Fraction(9, 128), Fraction(47, 64), Fraction(25, 128)]),
        (3, 5.625, 5, [Fraction(49, 128), Fraction(39, 64), Fraction(1, 128)]),
        (4, 2.0, 1, [Fraction(1, 6), Fraction(2, 3), Fraction(1, 6), Fraction(0)]),
        (4, 2.5, 1, [Fraction(1, 48), Fraction(23, 48), Fraction(23, 48), Fraction(1, 48)]),
    ]
    for order, u, first, exact in cases:
        cells, w = oracle.window_weights(np.array([u]), order)
        assert list(cells[0]) == list(range(first, first + order))
        np.testing.assert_allclose(w[0], [float(f) for f in exact], rtol=0, atol=1e-16)


def test_cic_node_particle_single_cell():
    n, box = 8, 100.0
    pos = np.array([[3 * box / n, 5 * box / n, 0.0]])
    mesh = oracle.paint_mesh(pos, n, box, 2)
    assert mesh[3, 5, 0] == 1.0
    assert np.count_nonzero(mesh) == 1


def _brute_paint(pos, w, n, box, order, shift):
    """Per particle, per cell: sum over periodic images of M_p(u - j - kN)."""
    mesh = np.zeros((n, n, n))
    for (x, y, z), wp in zip(pos, w):
        u = [float(c) % box * n / box + shift for c in (x, y, z)]
        f = []
        for d in range(3):
            f.append([sum(float(bspline(order, u[d] - j - k * n)) for k in (-1, 0, 1, 2))
                      for j in range(n)])
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    mesh[i, j, k] += wp * f[0][i] * f[1][j] * f[2][k]
    return mesh


@pytest.mark.parametrize("order,shift", [(2, 0.0), (3, 0.0), (4, 0.0), (2, 0.5), (3, 0.5)])
def test_paint_matches_brute_force(order, shift):
    n, box = 6, 10.0
    rng = np.random.default_rng(3 + order)
    pos = rng.uniform(-3, 13, (7, 3))  # also exercises the periodic wrap
    w = rng.uniform(0.5, 2.0, 7)
    got = oracle.paint_mesh(pos, n, box, order, weight=w, shift_cells=shift)
    want = _brute_paint(pos, w, n, box, order, shift)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_mass_conservation(order):
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 50.0, (5000, 3))
    w = rng.uniform(0.1, 3.0, 5000)
    mesh = oracle.paint_mesh(pos, 16, 50.0, order, weight=w, shift_cells=0.5)
    assert abs(mesh.sum() - w.sum()) <= 1e-12 * w.sum()


@pytest.mark.parametrize("order", [2, 3, 4])
def test_whole_cell_shift_permutes_mesh(order):
    n, box = 16, 32.0
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, box, (300, 3))
    a = oracle.paint_mesh(pos, n, box, order)
    shift = np.array([1, 2, 5]) * box / n
    b = oracle.paint_mesh(pos + shift, n, box, order)
    np.testing.assert_allclose(np.roll(a, (1, 2, 5), axis=(0, 1, 2)), b, atol=1e-12)


def test_wrap_handles_edges():
    box = 10.0
    x = np.array([-1e-17, 10.0, -10.0, 25.0, 9.999999999999998])
    got = oracle.wrap_positions(x, box)
    assert np.all(got >= 0) and np.all(got < box)
    np.testing.assert_allclose(got[:4], [0.0, 0.0, 0.0, 5.0])


@pytest.mark.parametrize("order,shift", [(2, 0.0), (3, 0.5), (4, 0.0)])
def test_paint_cells_matches_brute_force(order, shift):
    n, box = 6, 10.0
    rng = np.random.default_rng(40 + order)
    pos = rng.uniform(-3, 13, (9, 3))
    w = rng.uniform(0.5, 2.0, 9)
    want = _brute_paint(pos, w, n, box, order, shift)
    cells = rng.integers(0, n, (25, 3))
    got = oracle.paint_cells(pos, cells, n, box, order, weight=w, shift_cells=shift)
    np.testing.assert_allclose(got, want[cells[:, 0], cells[:, 1], cells[:, 2]], atol=1e-13)


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_painted_modes_equal_the_transform_of_the_painted_mesh(order, shift):
    # two independent routes to the same numbers: per-particle separable
    # sums against painting on the mesh followed by the float64 r2c
    n, box = 16, 50.0
    rng = np.random.default_rng(order * 10 + int(2 * shift))
    pos = rng.uniform(-box, 2 * box, (400, 3))  # also exercises the wrap
    w = rng.uniform(0.5, 1.5, 400)
    modes = np.stack([rng.integers(-7, 8, 40), rng.integers(-7, 8, 40),
                      rng.integers(0, 8, 40)], axis=1)
    modes[0] = (0, 0, 0)
    got = oracle.painted_modes(pos, modes, n, box, order, w, shift)
    c = oracle.r2c(oracle.paint_mesh(pos, n, box, order, w, shift))
    want = c[modes[:, 0] % n, modes[:, 1] % n, modes[:, 2]]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-10)
    assert got[0].real == pytest.approx(w.sum(), rel=1e-12)  # DC = sum of weights
