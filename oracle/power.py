"""Oracle: r2c transform, interlacing, compensation and the FFTPower binning.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Paper passages followed
-----------------------
* Sec. 3.3.1: RealField and ComplexField are related by a real-to-complex FFT
  (r2c).  Reading: forward transform with exp(-i k.x), no 1/N^3 factor
  (the scale is folded into the power normalisation).
* Sec. 3.3.2, interlacing: two meshes half a cell apart are combined in
  Fourier space.  Reading: c = (c_A + exp(+i k.s) c_B) / 2 with s = H/2 on
  every axis and k taken from the signed FFT index, i.e. the phase is
  exp(i pi (n_x + n_y + n_z) / N).
* Sec. 3.3.2, Eq. (2): compensation divides by prod_i sinc^p(pi k_i / 2 k_N)
  with k_N = pi N / L, i.e. sinc^p(pi n_i / N) for integer mode n_i.
* Sec. 3.4.1 (FFTPower): P(k), P(k, mu) and the multipoles P_ell(k) from
  |delta(k)|^2, mu the cosine to the line of sight.

Readings where the paper is silent (all pinned by tests):
* delta~ = DFT(F) / sum(w), P = V |delta~|^2 (the mesh holds 1 + delta
  up to the factor N^3 / sum(w));
* k-bins are half-open [e_b, e_{b+1}) with e_b = kmin + b dk in units of the
  fundamental k_f = 2 pi / L, decided on the integer n^2 against float64 e_b^2;
  the DC mode is excluded and the top edge is exclusive;
* mu is folded to |mu| in [0, 1] with Nmu equal bins; the bin is the largest j
  with j^2 n^2 <= Nmu^2 n_los^2 (exact integers), clipped to Nmu - 1 so that
  |mu| = 1 lands in the last bin;
* modes on the r2c half grid carry the Hermitian weight h = 1 on the
  n_z = 0 and n_z = N/2 planes and h = 2 elsewhere, so that counts equal a
  full-grid enumeration;
* P_ell = (2 ell + 1) x mode average of P L_ell(mu); shot noise
  V sum(w^2) / sum(w)^2 is reported and not subtracted; empty bins are NaN.
* value painting (Sec. 3.3.1: F = [1 + delta'] V with the weighted
  overdensity delta'): each particle paints w V, the normalisation stays
  sum(w), and the reported shot noise becomes V sum((w V)^2) / sum(w)^2, the
  Poisson noise of the painted field;
* cross power of two fields on one mesh: P_12 = V Re(c_1 conj(c_2)) /
  (W_1 W_2), binned like P; its shot noise (distinct catalogs) is zero.
* projected power (ProjectedFFTPower, Sec. 3.4.1): the painted field is
  summed over the projected axes, the d kept axes are transformed, and
  P = L^d |c|^2 / (sum w)^2 is binned in |k| over the kept axes (every mode
  of the full d-dimensional grid once); interlacing and compensation act on
  the kept axes (the projected ones have n = 0).  Shot noise L^d sum w^2 /
  (sum w)^2.
"""

import os

import numpy as np
import scipy.fft

from .paint import WINDOW_ORDER, paint_mesh


def r2c(mesh, workers=None):
    """Forward real-to-complex 3D DFT, exp(-i k.x), unnormalised (float64)."""
    if workers is None:
        workers = os.cpu_count()
    return scipy.fft.rfftn(np.asarray(mesh, dtype=np.float64), workers=workers)


def c2r(cmesh, nmesh, workers=None):
    """Backward complex-to-real 3D DFT, exp(+i k.x), unnormalised (float64):
    the full-grid sum over the Hermitian spectrum whose half is ``cmesh``
    (N, N, N/2 + 1), so that c2r(r2c(F)) = N^3 F."""
    if workers is None:
        workers = os.cpu_count()
    n = int(nmesh)
    return scipy.fft.irfftn(np.asarray(cmesh, dtype=np.complex128), s=(n, n, n),
                            workers=workers) * float(n) ** 3


def mode_indices(nmesh):
    """Signed integer wave numbers of the r2c array (numpy fftfreq order).

    Axis x and y: n = i for i < N/2, else i - N.  Axis z (the halved axis):
    n = i for i = 0 .. N/2.
    """
    full = np.arange(nmesh, dtype=np.int64)
    full = np.where(full < nmesh // 2, full, full - nmesh)
    half = np.arange(nmesh // 2 + 1, dtype=np.int64)
    return full, full.copy(), half


def interlace_combine(c_a, c_b, nmesh):
    """c = (c_A + exp(i pi (n_x + n_y + n_z) / N) c_B) / 2   (Sec. 3.3.2)."""
    nx, ny, nz = mode_indices(nmesh)
    s = nx[:, None, None] + ny[None, :, None] + nz[None, None, :]
    phase = np.exp(1j * np.pi * s / nmesh)
    return 0.5 * (c_a + phase * c_b)


def _sinc(x):
    """sinc(x) = sin(x) / x with sinc(0) = 1 (the paper's definition)."""
    x = np.asarray(x, dtype=np.float64)
    safe = np.where(x == 0.0, 1.0, x)
    return np.where(x == 0.0, 1.0, np.sin(safe) / safe)


def compensate(c, nmesh, order):
    """c / prod_d sinc^p(pi n_d / N)   (Eq. 2, pi k / 2 k_N = pi n / N)."""
    nx, ny, nz = mode_indices(nmesh)
    wx = _sinc(np.pi * nx / nmesh) ** order
    wy = _sinc(np.pi * ny / nmesh) ** order
    wz = _sinc(np.pi * nz / nmesh) ** order
    return c / (wx[:, None, None] * wy[None, :, None] * wz[None, None, :])


def kbin_edges_sq(kmin_f, dk_f, nk):
    """Squared bin edges e_b^2, e_b = kmin + b dk (units of k_f), b = 0..nk."""
    b = np.arange(nk + 1, dtype=np.float64)
    e = kmin_f + b * dk_f
    return e * e


def kbin_index(n2, edges_sq):
    """Largest b with e_b^2 <= n^2; -1 for the DC mode and out-of-range modes."""
    n2 = np.asarray(n2, dtype=np.int64)
    nk = len(edges_sq) - 1
    b = np.searchsorted(edges_sq, n2.astype(np.float64), side="right") - 1
    bad = (n2 == 0) | (b < 0) | (b >= nk)
    return np.where(bad, -1, b)


def _isqrt(v):
    """Exact integer square root of non-negative int64 values below 2^52."""
    v = np.asarray(v, dtype=np.int64)
    r = np.floor(np.sqrt(v.astype(np.float64))).astype(np.int64)
    r = np.where(r * r > v, r - 1, r)
    r = np.where((r + 1) * (r + 1) <= v, r + 1, r)
    return r


def mubin_index(nlos2, n2, nmu):
    """Largest j in [0, Nmu] with j^2 n^2 <= Nmu^2 n_los^2, clipped to Nmu - 1.

    Since j^2 is an integer, j^2 n^2 <= X is the same as j^2 <= floor(X / n^2),
    so j = isqrt(floor(Nmu^2 n_los^2 / n^2)) in exact integer arithmetic.
    Requires n^2 > 0.
    """
    nlos2 = np.asarray(nlos2, dtype=np.int64)
    n2 = np.asarray(n2, dtype=np.int64)
    j = _isqrt((nmu * nmu * nlos2) // n2)
    return np.minimum(j, nmu - 1)


def legendre(ell, mu2):
    """Legendre polynomial L_ell(mu) for even ell, as a function of mu^2."""
    if ell == 0:
        return np.ones_like(mu2)
    if ell == 2:
        return (3.0 * mu2 - 1.0) / 2.0
    if ell == 4:
        return (35.0 * mu2 * mu2 - 30.0 * mu2 + 3.0) / 8.0
    if ell == 6:
        return (231.0 * mu2 ** 3 - 315.0 * mu2 * mu2 + 105.0 * mu2 - 5.0) / 16.0
    raise ValueError("ell must be one of 0, 2, 4, 6")


def _check_bins(nmesh, interlaced, kmin_f, dk_f, nk, nmu, poles, los):
    if nk < 1 or dk_f <= 0 or kmin_f < 0:
        raise ValueError("need nk >= 1, dk > 0, kmin >= 0")
    if interlaced and kmin_f + nk * dk_f > nmesh // 2:
        raise ValueError("interlaced: the top edge may not exceed the Nyquist index")
    if any(ell % 2 for ell in poles):
        raise ValueError("only even multipoles")
    if los not in (0, 1, 2):
        raise ValueError("los is an axis index 0, 1 or 2")


def _accumulate(nmesh, kmin_f, dk_f, nk, nmu, poles, los, power_of_plane, slab):
    """Sum h, h|k|, h P, h P L_ell over k-bins and h, h|k|, h|mu|, h P over
    (k, mu)-bins, one slab of x-planes at a time.  ``power_of_plane(x0, x1)``
    returns the per-mode power of planes x0..x1-1 (or None for tables only).
    """
    n = nmesh
    nx, ny, nz = mode_indices(n)
    e2 = kbin_edges_sq(kmin_f, dk_f, nk)
    h_z = np.where((nz == 0) | (nz == n // 2), 1, 2).astype(np.int64)
    out = {
        "modes": np.zeros(nk, dtype=np.int64),
        "sum_k": np.zeros(nk),
        "sum_p": np.zeros(nk),
        "sum_pl": {ell: np.zeros(nk) for ell in poles},
    }
    use2d = nmu > 1
    if use2d:
        out.update(
            modes2d=np.zeros(nk * nmu, dtype=np.int64),
            sum_k2d=np.zeros(nk * nmu),
            sum_mu2d=np.zeros(nk * nmu),
            sum_p2d=np.zeros(nk * nmu),
        )
    for x0 in range(0, n, slab):
        x1 = min(n, x0 + slab)
        gx = nx[x0:x1, None, None]
        gy = ny[None, :, None]
        gz = nz[None, None, :]
        n2 = gx * gx + gy * gy + gz * gz
        shape = n2.shape
        n2 = n2.ravel()
        h = np.broadcast_to(h_z[None, None, :], shape).ravel()
        nlos = (gx, gy, gz)[los]
        nlos2 = np.broadcast_to(nlos * nlos, shape).ravel()
        b = kbin_index(n2, e2)
        sel = b >= 0
        b = b[sel]
        n2s = n2[sel]
        hs = h[sel].astype(np.float64)
        kabs = np.sqrt(n2s.astype(np.float64))  # in units of k_f
        mu2 = nlos2[sel].astype(np.float64) / n2s.astype(np.float64)
        out["modes"] += np.bincount(b, weights=h[sel], minlength=nk).astype(np.int64)
        out["sum_k"] += np.bincount(b, weights=hs * kabs, minlength=nk)
        p = None
        if power_of_plane is not None:
            p = power_of_plane(x0, x1).ravel()[sel]
            hp = hs * p
            out["sum_p"] += np.bincount(b, weights=hp, minlength=nk)
            for ell in poles:
                out["sum_pl"][ell] += np.bincount(
                    b, weights=hp * legendre(ell, mu2), minlength=nk
                )
        if use2d:
            j = mubin_index(nlos2[sel], n2s, nmu)
            f = b * nmu + j
            m = nk * nmu
            out["modes2d"] += np.bincount(f, weights=h[sel], minlength=m).astype(np.int64)
            out["sum_k2d"] += np.bincount(f, weights=hs * kabs, minlength=m)
            out["sum_mu2d"] += np.bincount(f, weights=hs * np.sqrt(mu2), minlength=m)
            if p is not None:
                out["sum_p2d"] += np.bincount(f, weights=hp, minlength=m)
    return out


def _slab(nmesh):
    return max(1, min(nmesh, (1 << 22) // (nmesh * (nmesh // 2 + 1))))


def mode_tables(nmesh, boxsize, kmin_f=0.0, dk_f=1.0, nk=None, nmu=0, los=2,
                interlaced=False):
    """Field-independent per-bin tables: counts, mean |k| and mean |mu|."""
    if nk is None:
        nk = nmesh // 2
    _check_bins(nmesh, interlaced, kmin_f, dk_f, nk, nmu, (), los)
    acc = _accumulate(nmesh, kmin_f, dk_f, nk, nmu, (), los, None, _slab(nmesh))
    kf = 2.0 * np.pi / boxsize
    with np.errstate(invalid="ignore", divide="ignore"):
        res = {"modes": acc["modes"], "k": kf * acc["sum_k"] / acc["modes"]}
        if nmu > 1:
            res["modes2d"] = acc["modes2d"].reshape(nk, nmu)
            res["k2d"] = (kf * acc["sum_k2d"] / acc["modes2d"]).reshape(nk, nmu)
            res["mu2d"] = (acc["sum_mu2d"] / acc["modes2d"]).reshape(nk, nmu)
    return res


def fftpower_from_spectra(c_a, c_b, nmesh, boxsize, order, compensated, wsum,
                          w2sum, npart, kmin_f=0.0, dk_f=1.0, nk=None, nmu=0,
                          poles=(), los=2):
    """FFTPower binning from the r2c spectra of mesh A (and B if interlaced).

    Follows Sec. 3.4.1 with the steps: interlace (Sec. 3.3.2), compensate
    (Eq. 2), P = V |c|^2 / (sum w)^2, then the k / mu / Legendre binning.
    """
    n = nmesh
    interlaced = c_b is not None
    if nk is None:
        nk = n // 2
    _check_bins(n, interlaced, kmin_f, dk_f, nk, nmu, poles, los)
    c = interlace_combine(c_a, c_b, n) if interlaced else np.asarray(c_a)
    if compensated:
        c = compensate(c, n, order)
    volume = float(boxsize) ** 3
    pmode = volume * (c.real ** 2 + c.imag ** 2) / (wsum * wsum)
    acc = _accumulate(n, kmin_f, dk_f, nk, nmu, tuple(poles), los,
                      lambda x0, x1: pmode[x0:x1], _slab(n))
    kf = 2.0 * np.pi / boxsize
    with np.errstate(invalid="ignore", divide="ignore"):
        nb = acc["modes"]
        res = {
            "k": kf * acc["sum_k"] / nb,
            "power": acc["sum_p"] / nb,
            "modes": nb,
            "poles": {ell: (2 * ell + 1) * acc["sum_pl"][ell] / nb for ell in poles},
            "shotnoise": volume * w2sum / (wsum * wsum),
            "wsum": wsum,
            "w2sum": w2sum,
            "npart": npart,
            "edges": kf * (kmin_f + dk_f * np.arange(nk + 1)),
        }
        if nmu > 1:
            m2 = acc["modes2d"]
            res["modes2d"] = m2.reshape(nk, nmu)
            res["k2d"] = (kf * acc["sum_k2d"] / m2).reshape(nk, nmu)
            res["mu2d"] = (acc["sum_mu2d"] / m2).reshape(nk, nmu)
            res["power2d"] = (acc["sum_p2d"] / m2).reshape(nk, nmu)
    return res


def fftpower(pos, nmesh, boxsize, window="cic", interlaced=False,
             compensated=True, weight=None, kmin_f=0.0, dk_f=1.0, nk=None,
             nmu=0, poles=(), los=2, workers=None, value=None):
    """End-to-end oracle FFTPower on a periodic box (Sec. 3.3 and 3.4.1).
    ``value``: per-particle field value V (Sec. 3.3.1), painted as w V."""
    order = WINDOW_ORDER[window] if isinstance(window, str) else int(window)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    wv = w if value is None else w * np.asarray(value, dtype=np.float64)
    wsum = float(np.sum(w))
    w2sum = float(np.sum(wv * wv))
    c_a = r2c(paint_mesh(pos, nmesh, boxsize, order, wv), workers)
    c_b = None
    if interlaced:
        c_b = r2c(paint_mesh(pos, nmesh, boxsize, order, wv, 0.5), workers)
    return fftpower_from_spectra(c_a, c_b, nmesh, boxsize, order, compensated,
                                 wsum, w2sum, len(pos), kmin_f, dk_f, nk, nmu,
                                 poles, los)


def prepared_spectrum(pos, nmesh, boxsize, window="cic", interlaced=False,
                      compensated=True, weight=None, workers=None):
    """The spectrum of one catalog after interlacing and compensation
    (Sec. 3.3.2, Eq. 2) and its sum of weights: the input of a cross power."""
    order = WINDOW_ORDER[window] if isinstance(window, str) else int(window)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    c = r2c(paint_mesh(pos, nmesh, boxsize, order, w), workers)
    if interlaced:
        c = interlace_combine(c, r2c(paint_mesh(pos, nmesh, boxsize, order, w, 0.5), workers),
                              nmesh)
    if compensated:
        c = compensate(c, nmesh, order)
    return c, float(np.sum(w))


def cross_from_spectra(c1, c2, nmesh, boxsize, wsum1, wsum2, kmin_f=0.0, dk_f=1.0, nk=None,
                       nmu=0, poles=(), los=2, interlaced=False):
    """Cross power of two prepared spectra: per mode V Re(c1 conj(c2)) /
    (W1 W2), binned exactly like the auto power (Sec. 3.4.1)."""
    n = nmesh
    if nk is None:
        nk = n // 2
    _check_bins(n, interlaced, kmin_f, dk_f, nk, nmu, poles, los)
    volume = float(boxsize) ** 3
    pmode = volume * (c1.real * c2.real + c1.imag * c2.imag) / (wsum1 * wsum2)
    acc = _accumulate(n, kmin_f, dk_f, nk, nmu, tuple(poles), los,
                      lambda x0, x1: pmode[x0:x1], _slab(n))
    kf = 2.0 * np.pi / boxsize
    with np.errstate(invalid="ignore", divide="ignore"):
        nb = acc["modes"]
        res = {
            "k": kf * acc["sum_k"] / nb,
            "power": acc["sum_p"] / nb,
            "modes": nb,
            "poles": {ell: (2 * ell + 1) * acc["sum_pl"][ell] / nb for ell in poles},
            "shotnoise": 0.0,
            "wsum": float(np.sqrt(wsum1 * wsum2)),
            "w2sum": 0.0,
        }
        if nmu > 1:
            m2 = acc["modes2d"]
            res["modes2d"] = m2.reshape(nk, nmu)
            res["k2d"] = (kf * acc["sum_k2d"] / m2).reshape(nk, nmu)
            res["mu2d"] = (acc["sum_mu2d"] / m2).reshape(nk, nmu)
            res["power2d"] = (acc["sum_p2d"] / m2).reshape(nk, nmu)
    return res


def projected_power(pos, nmesh, boxsize, keep, window="cic", interlaced=False,
                    compensated=True, weight=None, kmin_f=0.0, dk_f=1.0, nk=None):
    """ProjectedFFTPower of a periodic box: power of the field projected
    along the axes not in ``keep`` (a tuple of one or two axes)."""
    keep = tuple(sorted(int(a) for a in keep))
    if not 1 <= len(keep) <= 2 or any(a not in (0, 1, 2) for a in keep):
        raise ValueError("keep must hold one or two distinct axes")
    drop = tuple(a for a in range(3) if a not in keep)
    d = len(keep)
    n = nmesh
    if nk is None:
        nk = n // 2
    order = WINDOW_ORDER[window] if isinstance(window, str) else int(window)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.ones(len(pos)) if weight is None else np.asarray(weight, dtype=np.float64)
    wsum = float(np.sum(w))
    w2sum = float(np.sum(w * w))

    def spectrum(shift):
        proj = paint_mesh(pos, n, boxsize, order, w, shift).sum(axis=drop)
        return np.fft.fftn(proj)  # full d-dimensional grid, exp(-i k.x)

    c = spectrum(0.0)
    full = np.arange(n, dtype=np.int64)
    full = np.where(full < n // 2, full, full - n)
    grids = np.meshgrid(*([full] * d), indexing="ij")
    if interlaced:
        s = sum(grids)
        c = 0.5 * (c + np.exp(1j * np.pi * s / n) * spectrum(0.5))
    if compensated:
        for g in grids:
            c = c / _sinc(np.pi * g / n) ** order
    n2 = sum(g * g for g in grids).ravel()
    area = float(boxsize) ** d
    pmode = (area * (c.real ** 2 + c.imag ** 2) / (wsum * wsum)).ravel()
    b = kbin_index(n2, kbin_edges_sq(kmin_f, dk_f, nk))
    sel = b >= 0
    cnt = np.bincount(b[sel], minlength=nk).astype(np.int64)
    sk = np.bincount(b[sel], weights=np.sqrt(n2[sel].astype(np.float64)), minlength=nk)
    sp = np.bincount(b[sel], weights=pmode[sel], minlength=nk)
    kf = 2.0 * np.pi / boxsize
    with np.errstate(invalid="ignore", divide="ignore"):
        return {"k": kf * sk / cnt, "power": sp / cnt, "modes": cnt, "poles": {},
                "shotnoise": area * w2sum / (wsum * wsum), "wsum": wsum, "w2sum": w2sum}
