"""Oracle: painting a catalog onto a periodic mesh (float64, CPU).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Paper passages followed
-----------------------
* Sec. 3.3.1, Eq. (1): the painted field is F(x) = [1 + delta'(x)] V(x) with
  n'(x) = W(x) n(x); in the default case W = V = 1 and F is 1 + delta.  Here
  the mesh holds the weighted sum of window values, F_j = sum_p w_p W(u_p - j);
  the division by sum(w) that turns it into 1 + delta is folded into the power
  normalisation (``power.py``).
* Sec. 3.3.2: the CIC, TSC and PCS windows.  The paper fixes them through the
  sinc^p compensation of Eq. (2) with p = 2, 3, 4; the only window whose
  Fourier transform is sinc^p is the centred cardinal B-spline of order p
  (p-fold self-convolution of the unit box), which is what ``bspline`` below
  evaluates.
* Sec. 3.3.2 (interlacing): the second mesh is offset by half a cell; it is
  painted here from u + 1/2 (``shift_cells = 0.5``).

Readings where the paper is silent (each one is pinned by a test):
* mesh nodes sit at x = j H, H = L / N, so the cell coordinate is u = x N / L;
* positions outside [0, L) wrap periodically;
* TSC rounds its centre cell as floor(u + 1/2) (the weights are continuous,
  so the tie choice does not change the result).
"""

import numpy as np

WINDOW_ORDER = {"cic": 2, "tsc": 3, "pcs": 4}


def wrap_positions(pos, boxsize):
    """Periodic wrap of positions into [0, L) (reading: positions wrap)."""
    x = np.asarray(pos, dtype=np.float64)
    x = x - boxsize * np.floor(x / boxsize)
    # x / L can round so that a tiny negative x lands exactly on L.
    x = np.where(x >= boxsize, 0.0, x)
    return x


def cell_coordinates(pos, nmesh, boxsize):
    """u = x N / L for wrapped positions: mesh node j sits at u = j."""
    return wrap_positions(pos, boxsize) * nmesh / boxsize


def bspline(order, a):
    """Centred cardinal B-spline M_p(a) of order p = 2, 3, 4 (Sec. 3.3.2).

    M_2 is the CIC tent, M_3 the TSC quadratic, M_4 the PCS cubic.  Each is
    the p-fold convolution of the unit box on [-1/2, 1/2].
    """
    a = np.abs(np.asarray(a, dtype=np.float64))
    if order == 2:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if order == 3:
        return np.where(
            a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0)
        )
    if order == 4:
        return np.where(
            a < 1.0,
            (4.0 - 6.0 * a * a + 3.0 * a ** 3) / 6.0,
            np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0),
        )
    raise ValueError("window order must be 2 (CIC), 3 (TSC) or 4 (PCS)")


def window_weights(u, order):
    """Cells and weights of the order-p window for cell coordinates u.

    Returns ``(cells, weights)``, each of shape ``u.shape + (p,)``: the p
    (unwrapped) integer cells that the window touches and M_p(u - j) there.
    Even orders start from floor(u); odd orders centre on floor(u + 1/2).
    """
    u = np.asarray(u, dtype=np.float64)
    if order % 2 == 0:
        first = np.floor(u) - (order // 2 - 1)
    else:
        first = np.floor(u + 0.5) - (order - 1) // 2
    offsets = np.arange(order, dtype=np.float64)
    cells = first[..., None] + offsets
    weights = bspline(order, u[..., None] - cells)
    return cells.astype(np.int64), weights


def paint_mesh(pos, nmesh, boxsize, order, weight=None, shift_cells=0.0):
    """F_j = sum_p w_p prod_d M_p(u_{p,d} + shift - j_d), periodic (Eq. 1).

    ``pos`` is (N_p, 3) in the box units, ``weight`` is (N_p,) or None for
    unit weights, ``shift_cells`` is 0 for the plain mesh and 1/2 for the
    interlaced mesh.  Returns a float64 (N, N, N) array indexed [x, y, z].
    Each of the p^3 stencil offsets is accumulated with ``np.bincount``, a
    sequential float64 sum.
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = nmesh
    u = cell_coordinates(pos, n, boxsize) + shift_cells
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    cx, wx = window_weights(u[:, 0], order)
    cy, wy = window_weights(u[:, 1], order)
    cz, wz = window_weights(u[:, 2], order)
    cx %= n
    cy %= n
    cz %= n
    mesh = np.zeros(n ** 3, dtype=np.float64)
    for a in range(order):
        for b in range(order):
            for c in range(order):
                flat = (cx[:, a] * n + cy[:, b]) * n + cz[:, c]
                mesh += np.bincount(
                    flat, weights=w * wx[:, a] * wy[:, b] * wz[:, c], minlength=n ** 3
                )
    return mesh.reshape(n, n, n)


def paint_cells(pos, cells, nmesh, boxsize, order, weight=None, shift_cells=0.0):
    """F_j of Eq. (1) at the listed cells only, one cell at a time.

    For each cell j = (i, k, l) this sums w_p prod_d M_p(u_{p,d} + shift - j_d
    - m_d N) over all particles, with m_d the periodic image nearest to the
    cell (for N >= p no other image is within the window's reach).  Used to
    check single cells of meshes too large to paint on the host.
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    u = cell_coordinates(pos, nmesh, boxsize) + shift_cells
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    out = np.empty(len(cells))
    reach = order / 2.0
    for c, cell in enumerate(np.asarray(cells, dtype=np.int64).reshape(-1, 3)):
        total = w.copy()
        for d in range(3):
            a = u[:, d] - cell[d]
            a = a - nmesh * np.round(a / nmesh)  # nearest periodic image
            total = total * np.where(np.abs(a) < reach, bspline(order, a), 0.0)
        out[c] = total.sum()
    return out


def painted_modes(pos, modes, nmesh, boxsize, order, weight=None, shift_cells=0.0):
    """DFT of the painted mesh, c(n) = sum_j F_j exp(-2 pi i n.j / N), at the
    listed integer modes only, without forming the mesh.

    F_j is a sum over particles of a product of one window per axis, so each
    particle contributes prod_d sum_{cells j_d} M_p(u_d - j_d)
    exp(-2 pi i n_d j_d / N): a few terms per axis and particle.  The
    exponential is periodic in j_d, so the cells need no wrapping.  Used to
    check modes of meshes too large to transform on the host.  Returns a
    complex128 array, one value per row of ``modes``.
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 3)
    u = cell_coordinates(pos, nmesh, boxsize) + shift_cells
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    # per axis, the factor of every particle for every distinct n_d needed;
    # exp(-2 pi i n_d j / N) is the |n_d|-th power of the n_d = 1 phase
    # (conjugated for n_d < 0)
    factors = []
    for d in range(3):
        cells, wts = window_weights(u[:, d], order)
        base = np.exp(-2j * np.pi * cells / nmesh)
        table = {}
        for nd in np.unique(modes[:, d]):
            nd = int(nd)
            phase = np.ones_like(base)
            for _ in range(abs(nd)):
                phase = phase * base
            if nd < 0:
                phase = np.conj(phase)
            table[nd] = np.sum(wts * phase, axis=1)
        factors.append(table)
    out = np.empty(len(modes), dtype=np.complex128)
    for i, (nx, ny, nz) in enumerate(modes):
        out[i] = np.sum(w * factors[0][int(nx)] * factors[1][int(ny)] * factors[2][int(nz)])
    return out
