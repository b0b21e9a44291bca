"""Oracle: survey power-spectrum multipoles (ConvolvedFFTPower, Sec. 3.4.1).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper names the estimator (the FFT-based multipoles of Hand et al. 2017,
which need 2 ell + 1 FFTs for a multipole ell) without spelling it out, so
the definitions below are the standard ones of that estimator, written from
their mathematics; parity with the paper itself is unpinned.  They are
pinned here against exact identities: the addition theorem of the real
spherical harmonics, a brute-force evaluation of F_ell on a tiny mesh, and the
limit of a distant observer, where the estimator reduces to the FFTPower
multipoles along the line of sight.

Definitions (box coordinates x wrapped into [0, L) as for the painting,
observer o, r = x - o, r^ = r / |r|, r^ = z^ where r = 0; reading: the line
of sight of a particle is taken at its position in the periodic box, which
is the position as given for a survey embedded in the box):
* weighted field F(x) = sum_data w delta_D(x - x_i) - alpha sum_randoms w
  delta_D(x - x_j), alpha = sum_data w / sum_randoms w;
* A_lm(k) = DFT of the mesh painted with w s Y_lm(r^) (s = 1 for data,
  -alpha for randoms), compensated by the window like FFTPower (Eq. 2);
* F_ell(k) = 4 pi / (2 ell + 1) sum_m Y_lm(k^) A_lm(k), with real orthonormal
  spherical harmonics; by the addition theorem this is the transform of
  sum_i w_i s_i L_ell(k^ . r^_i) painted;
* P_ell(k) = (2 ell + 1) / I x shell average of Re[F_0(k) conj F_ell(k)],
  I the normalisation (an input: it depends on the survey's mean density);
  shot noise (sum_data w^2 + alpha^2 sum_randoms w^2) / I, reported, not
  subtracted.  Modes with |n| >= N/2 are not binned (top edge <= N/2).
"""

import math

import numpy as np

from .paint import WINDOW_ORDER, paint_mesh, wrap_positions
from .power import (_accumulate, _check_bins, _slab, compensate, mode_indices, r2c)


def real_ylm(ell, m, x, y, z):
    """Real orthonormal spherical harmonic Y_lm at unit vectors (x, y, z),
    ell in {0, 2, 4}, -ell <= m <= ell (m < 0: the sine-type harmonics)."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    pi = math.pi
    if ell == 0:
        return np.full(np.broadcast(x, y, z).shape, 0.5 / math.sqrt(pi))
    if ell == 2:
        table = {
            -2: 0.5 * math.sqrt(15 / pi) * x * y,
            -1: 0.5 * math.sqrt(15 / pi) * y * z,
            0: 0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),
            1: 0.5 * math.sqrt(15 / pi) * x * z,
            2: 0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        }
        return table[m]
    if ell == 4:
        x2, y2, z2 = x * x, y * y, z * z
        table = {
            -4: 0.75 * math.sqrt(35 / pi) * x * y * (x2 - y2),
            -3: 0.75 * math.sqrt(35 / (2 * pi)) * y * z * (3 * x2 - y2),
            -2: 0.75 * math.sqrt(5 / pi) * x * y * (7 * z2 - 1),
            -1: 0.75 * math.sqrt(5 / (2 * pi)) * y * z * (7 * z2 - 3),
            0: 3 / 16 * math.sqrt(1 / pi) * (35 * z2 * z2 - 30 * z2 + 3),
            1: 0.75 * math.sqrt(5 / (2 * pi)) * x * z * (7 * z2 - 3),
            2: 3 / 8 * math.sqrt(5 / pi) * (x2 - y2) * (7 * z2 - 1),
            3: 0.75 * math.sqrt(35 / (2 * pi)) * x * z * (x2 - 3 * y2),
            4: 3 / 16 * math.sqrt(35 / pi) * (x2 * (x2 - 3 * y2) - y2 * (3 * x2 - y2)),
        }
        return table[m]
    raise ValueError("ell must be 0, 2 or 4")


def unit_vectors(pos, observer):
    """r^ of positions relative to the observer; z^ where r = 0."""
    r = np.asarray(pos, dtype=np.float64) - np.asarray(observer, dtype=np.float64)
    norm = np.sqrt(np.sum(r * r, axis=1))
    safe = np.where(norm > 0, norm, 1.0)
    out = r / safe[:, None]
    out[norm == 0] = (0.0, 0.0, 1.0)
    return out


def k_unit_vectors(nmesh):
    """k^ of the r2c modes (zeros at the DC mode)."""
    nx, ny, nz = mode_indices(nmesh)
    kx = nx[:, None, None] * np.ones((1, nmesh, nmesh // 2 + 1))
    ky = ny[None, :, None] * np.ones((nmesh, 1, nmesh // 2 + 1))
    kz = nz[None, None, :] * np.ones((nmesh, nmesh, 1))
    kn = np.sqrt(kx * kx + ky * ky + kz * kz)
    kn[0, 0, 0] = 1.0
    return kx / kn, ky / kn, kz / kn


def multipole_fields(data, randoms, w_data, w_rand, observer, nmesh, boxsize, window,
                     poles, compensated=True):
    """F_ell(k) for each ell in poles (dict), alpha and the weight sums."""
    order = WINDOW_ORDER[window] if isinstance(window, str) else int(window)
    wd = np.ones(len(data)) if w_data is None else np.asarray(w_data, dtype=np.float64)
    wr = np.ones(len(randoms)) if w_rand is None else np.asarray(w_rand, dtype=np.float64)
    alpha = float(wd.sum() / wr.sum())
    ud = unit_vectors(wrap_positions(data, boxsize), observer)
    ur = unit_vectors(wrap_positions(randoms, boxsize), observer)
    khat = k_unit_vectors(nmesh)
    fields = {}
    for ell in poles:
        f = np.zeros((nmesh, nmesh, nmesh // 2 + 1), dtype=np.complex128)
        for m in range(-ell, ell + 1):
            mesh = paint_mesh(data, nmesh, boxsize, order, wd * real_ylm(ell, m, *ud.T))
            mesh -= paint_mesh(randoms, nmesh, boxsize, order,
                               alpha * wr * real_ylm(ell, m, *ur.T))
            a = r2c(mesh)
            if compensated:
                a = compensate(a, nmesh, order)
            f += real_ylm(ell, m, *khat) * a
        fields[ell] = 4 * math.pi / (2 * ell + 1) * f
    sums = {"wsum_data": float(wd.sum()), "w2sum_data": float((wd * wd).sum()),
            "wsum_rand": float(wr.sum()), "w2sum_rand": float((wr * wr).sum())}
    return fields, alpha, sums


def convolved_power(data, randoms, w_data, w_rand, observer, nmesh, boxsize, norm,
                    window="cic", poles=(0, 2, 4), compensated=True, kmin_f=0.0, dk_f=1.0,
                    nk=None):
    """P_ell(k) of a survey embedded in a box (the estimator above)."""
    if nk is None:
        nk = nmesh // 2
    _check_bins(nmesh, True, kmin_f, dk_f, nk, 0, (), 2)
    fields, alpha, sums = multipole_fields(data, randoms, w_data, w_rand, observer, nmesh,
                                           boxsize, window, tuple(poles), compensated)
    if 0 not in fields:
        fields[0] = multipole_fields(data, randoms, w_data, w_rand, observer, nmesh, boxsize,
                                     window, (0,), compensated)[0][0]
    f0 = fields[0]
    kf = 2 * math.pi / boxsize
    out = {"poles": {}, "alpha": alpha, "norm": float(norm), **sums}
    for ell in poles:
        fl = fields[ell]
        pmode = (2 * ell + 1) * (f0.real * fl.real + f0.imag * fl.imag) / norm
        acc = _accumulate(nmesh, kmin_f, dk_f, nk, 0, (), 2, lambda x0, x1: pmode[x0:x1],
                          _slab(nmesh))
        with np.errstate(invalid="ignore", divide="ignore"):
            out["poles"][ell] = acc["sum_p"] / acc["modes"]
            out["modes"] = acc["modes"]
            out["k"] = kf * acc["sum_k"] / acc["modes"]
    out["shotnoise"] = (sums["w2sum_data"] + alpha * alpha * sums["w2sum_rand"]) / norm
    return out
