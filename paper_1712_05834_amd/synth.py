"""Seeded synthetic inputs: catalogs and fields for tests and benchmarks.

This module only draws inputs.  It holds none of the estimator's arithmetic
(no painting, no forward transform of a catalog, no binning); the GPU library
and the CPU oracle both consume the arrays it returns.  Random numbers come
from ``numpy.random.Generator(PCG64(seed))``; Gaussian fields are shaped with
SciPy's float64 FFTs.

Recipes (the nbodykit paper names the catalog types, Sec. 3.2: uniform random
columns and a Poisson-sampled log-normal field; Sec. 5 uses Gaussian
realisations of an input P(k) and a Zel'dovich-displaced lattice):

* ``uniform_catalog``: N positions U[0, L)^3.
* ``gaussian_field``: white noise w ~ N(0, 1) on the grid, DFT(delta) =
  DFT(w) sqrt(N^3 P(|k|) / V) with the DC mode zeroed, so that
  E|DFT(delta) / N^3|^2 = P / V.
* ``fixed_amplitude_field``: the same phases with |DFT| fixed to
  N^3 sqrt(P / V) and DC = N^3, a mean-one field whose measured power equals
  the mode average of P(|k|) exactly.
* ``lognormal_catalog``: delta_LN = exp(delta_G - sigma^2 / 2) - 1 with sigma^2
  the mesh variance of delta_G; per-cell counts ~ Poisson(nbar_cell (1 +
  delta_LN)); positions at the cell corner plus U[0, 1)^3 H, in cell order.
* ``zeldovich_lattice``: lattice q = i L / G, psi~ = i k delta~ / k^2 (DC and
  Nyquist planes of psi~ zeroed so psi is real), x = q + psi wrapped into
  [0, L).
* ``lognormal_catalog_device``: the log-normal recipe drawn on the GPU with
  torch's seeded device generator (a Philox4x32-10 counter-based stream) and
  float32 FFTs, for workloads of hundreds of mocks whose host generation would
  take minutes.  Not bit-identical to ``lognormal_catalog``; tests that need
  the oracle read the catalog back.
* ``mock_batch_sizes``: the particle counts and mesh sizes of a batch of
  mocks: N_i = round(10^U(lo, hi)), meshes cycling through a list.
* ``survey_catalog``: a survey-like geometry for the multipoles with a
  varying line of sight: the log-normal catalog and rand_factor times as many
  uniform randoms, both cut to the shell rmin <= |x - observer| < rmax.
"""

import os

import numpy as np
import scipy.fft


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def pk_lognormal_c2(k, amp=2.0e4):
    """P(k) = A k / (1 + (k / 0.02)^2)^1.4, A = 2e4 (log-normal mock workload)."""
    k = np.asarray(k, dtype=np.float64)
    return amp * k / (1.0 + (k / 0.02) ** 2) ** 1.4


def pk_zeldovich_c3(k, amp=10.0):
    """P(k) = A k^-1.5 exp(-(k / 0.5)^2), A = 10 (Zel'dovich lattice workload)."""
    k = np.asarray(k, dtype=np.float64)
    safe = np.where(k > 0, k, 1.0)
    return np.where(k > 0, amp * safe ** -1.5 * np.exp(-((safe / 0.5) ** 2)), 0.0)


def _kmag(nmesh, boxsize):
    full = np.fft.fftfreq(nmesh, d=1.0 / nmesh)
    half = np.arange(nmesh // 2 + 1, dtype=np.float64)
    kf = 2.0 * np.pi / boxsize
    k2 = full[:, None, None] ** 2 + full[None, :, None] ** 2 + half[None, None, :] ** 2
    return kf * np.sqrt(k2)


def uniform_catalog(npart, boxsize, seed, dtype=np.float64):
    """npart positions uniform in [0, L)^3, shape (npart, 3)."""
    pos = rng_for(seed).uniform(0.0, boxsize, size=(npart, 3))
    pos = pos.astype(dtype)
    # rounding to float32 can reach L exactly; keep inputs in [0, L)
    pos[pos >= boxsize] = 0
    return pos


def _white_noise_hat(nmesh, seed):
    w = rng_for(seed).standard_normal((nmesh, nmesh, nmesh))
    return scipy.fft.rfftn(w, workers=os.cpu_count())


def gaussian_field(nmesh, boxsize, pk, seed):
    """Real Gaussian field delta_G on an N^3 grid with spectrum P(k) (float64)."""
    what = _white_noise_hat(nmesh, seed)
    amp = np.sqrt(nmesh ** 3 * pk(_kmag(nmesh, boxsize)) / boxsize ** 3)
    what *= amp
    what[0, 0, 0] = 0.0
    return scipy.fft.irfftn(what, s=(nmesh,) * 3, workers=os.cpu_count())


def fixed_amplitude_field(nmesh, boxsize, pk, seed):
    """Mean-one real field F with |DFT(F)| = N^3 sqrt(P(|k|) / V) exactly."""
    what = _white_noise_hat(nmesh, seed)
    mag = np.abs(what)
    mag[mag == 0] = 1.0
    amp = nmesh ** 3 * np.sqrt(pk(_kmag(nmesh, boxsize)) / boxsize ** 3)
    x = what / mag * amp
    x[0, 0, 0] = nmesh ** 3
    return scipy.fft.irfftn(x, s=(nmesh,) * 3, workers=os.cpu_count())


def lognormal_catalog(nmesh, boxsize, pk, nbar_cell, seed, dtype=np.float32):
    """Poisson-sampled log-normal catalog, particles listed in cell order."""
    delta_g = gaussian_field(nmesh, boxsize, pk, seed)
    sigma2 = float(np.var(delta_g))
    lam = nbar_cell * np.exp(delta_g - 0.5 * sigma2)
    del delta_g
    rng = rng_for(seed + 7919)
    counts = rng.poisson(lam.ravel())
    del lam
    cells = np.repeat(np.arange(nmesh ** 3, dtype=np.int64), counts)
    ix, rem = np.divmod(cells, nmesh * nmesh)
    iy, iz = np.divmod(rem, nmesh)
    del cells, rem
    h = boxsize / nmesh
    off = rng.uniform(0.0, 1.0, size=(len(ix), 3))
    pos = np.empty((len(ix), 3), dtype=np.float64)
    pos[:, 0] = (ix + off[:, 0]) * h
    pos[:, 1] = (iy + off[:, 1]) * h
    pos[:, 2] = (iz + off[:, 2]) * h
    pos = pos.astype(dtype)
    pos[pos >= boxsize] = 0
    return pos


def zeldovich_lattice(ngrid, boxsize, pk, seed, dtype=np.float32):
    """Lattice of ngrid^3 particles displaced by the Zel'dovich field of P(k)."""
    what = _white_noise_hat(ngrid, seed)
    amp = np.sqrt(ngrid ** 3 * pk(_kmag(ngrid, boxsize)) / boxsize ** 3)
    dhat = what * amp
    del what, amp
    dhat[0, 0, 0] = 0.0
    kf = 2.0 * np.pi / boxsize
    full = np.fft.fftfreq(ngrid, d=1.0 / ngrid)
    half = np.arange(ngrid // 2 + 1, dtype=np.float64)
    kvec = (kf * full[:, None, None], kf * full[None, :, None], kf * half[None, None, :])
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    k2[0, 0, 0] = 1.0
    nyq = ngrid // 2
    h = boxsize / ngrid
    q = np.arange(ngrid, dtype=np.float64) * h
    pos = np.empty((ngrid, ngrid, ngrid, 3), dtype=np.float64)
    for d in range(3):
        psi_hat = 1j * kvec[d] * dhat / k2
        psi_hat[0, 0, 0] = 0.0
        psi_hat[nyq, :, :] = 0.0
        psi_hat[:, nyq, :] = 0.0
        psi_hat[:, :, nyq] = 0.0
        psi = scipy.fft.irfftn(psi_hat, s=(ngrid,) * 3, workers=os.cpu_count())
        del psi_hat
        shape = [1, 1, 1]
        shape[d] = ngrid
        pos[..., d] = q.reshape(shape) + psi
        del psi
    pos = pos.reshape(-1, 3)
    pos -= boxsize * np.floor(pos / boxsize)
    pos = pos.astype(dtype)
    pos[pos >= boxsize] = 0
    return pos


def uniform_weights(npart, seed, low=0.5, high=1.5, dtype=np.float64):
    """Per-particle weights U[low, high) for the weighted-painting tests."""
    return rng_for(seed).uniform(low, high, size=npart).astype(dtype)


def lognormal_catalog_device(nmesh, boxsize, pk, nbar_cell, seed, device="cuda",
                             dtype=None):
    """The log-normal recipe on the device; returns an (n, 3) torch tensor in
    cell order (float32 unless dtype is given)."""
    import torch

    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = int(nmesh)
    w = torch.randn((n, n, n), generator=g, device=device, dtype=torch.float32)
    what = torch.fft.rfftn(w)
    del w
    # the amplitude depends on the integer n^2 only: tabulate it on the host
    kf = 2.0 * np.pi / boxsize
    n2max = 3 * (n // 2) ** 2
    table = np.sqrt(n ** 3 * pk(kf * np.sqrt(np.arange(n2max + 1, dtype=np.float64)))
                    / boxsize ** 3)
    table = torch.from_numpy(table.astype(np.float32)).to(device)
    full = torch.fft.fftfreq(n, d=1.0 / n, device=device).round().to(torch.int64)
    half = torch.arange(n // 2 + 1, device=device, dtype=torch.int64)
    n2 = full[:, None, None] ** 2 + full[None, :, None] ** 2 + half[None, None, :] ** 2
    what = what * table[n2]
    del n2, table
    what[0, 0, 0] = 0
    delta = torch.fft.irfftn(what, s=(n, n, n))
    del what
    sigma2 = float(delta.double().var())
    lam = nbar_cell * torch.exp(delta - 0.5 * sigma2)
    del delta
    counts = torch.poisson(lam.reshape(-1), generator=g).to(torch.int64)
    del lam
    cells = torch.repeat_interleave(torch.arange(n ** 3, device=device, dtype=torch.int64), counts)
    del counts
    ix = cells // (n * n)
    iy = (cells // n) % n
    iz = cells % n
    del cells
    off = torch.rand((ix.numel(), 3), generator=g, device=device, dtype=torch.float64)
    h = boxsize / n
    pos = torch.stack([(ix + off[:, 0]) * h, (iy + off[:, 1]) * h, (iz + off[:, 2]) * h], dim=1)
    del ix, iy, iz, off
    pos = pos.to(dtype)
    pos[pos >= boxsize] = 0
    return pos.contiguous()


def mock_batch_sizes(count, seed, meshes=(128, 256, 512), lo=5.0, hi=7.0):
    """(npart_target, nmesh) per mock: N_i = round(10^U(lo, hi)), mesh i mod len."""
    u = rng_for(seed).uniform(lo, hi, size=count)
    return [(int(round(10.0 ** x)), int(meshes[i % len(meshes)])) for i, x in enumerate(u)]


def survey_catalog(nmesh, boxsize, pk, nbar_cell, seed, observer, rmin, rmax, rand_factor=5.0,
                   dtype=np.float64):
    """(data, randoms): log-normal data and uniform randoms (rand_factor times
    the box's data count) kept where rmin <= |x - observer| < rmax."""
    obs = np.asarray(observer, dtype=np.float64)

    def cut(pos):
        r = np.sqrt(np.sum((pos.astype(np.float64) - obs) ** 2, axis=1))
        return pos[(r >= rmin) & (r < rmax)]

    data = lognormal_catalog(nmesh, boxsize, pk, nbar_cell, seed, dtype=dtype)
    nrand = int(round(rand_factor * len(data)))
    rand = uniform_catalog(nrand, boxsize, seed + 104729, dtype=dtype)
    return np.ascontiguousarray(cut(data)), np.ascontiguousarray(cut(rand))
