"""Device-side generation of Gaussian fields with the library's kernels.

A Gaussian field of spectrum P(k) is white noise shaped in Fourier space:
delta_G = c2r(r2c(w) sqrt(N^3 P(|k|) / V)) / N^3 with the DC mode removed --
the recipe of the catalogs built from Gaussian fields (Sec. 3.2), run here as
pk_fft_r2c, pk_shape_spectrum and pk_fft_c2r on the device.  The random
numbers are an input (``noise``): the caller draws them, so that the same
draws can be given to any other implementation of the recipe.
"""

import math

import numpy as np

from . import _lib


def amplitude_table(nmesh, boxsize, pk):
    """sqrt(N^3 P(k) / V) / N^3 at k = k_f sqrt(n^2) for n^2 = 0 .. 3 (N/2)^2,
    DC set to zero (float64, host)."""
    n = int(nmesh)
    n2 = np.arange(3 * (n // 2) ** 2 + 1, dtype=np.float64)
    kf = 2.0 * math.pi / boxsize
    amp = np.sqrt(n ** 3 * np.asarray(pk(kf * np.sqrt(n2)), dtype=np.float64) / boxsize ** 3)
    amp /= float(n) ** 3
    amp[0] = 0.0
    return amp


def gaussian_field(ctx, noise, boxsize, pk):
    """delta_G on the device from white noise: ``noise`` is an (N, N, N) CUDA
    tensor of float32 or float64, N a power of two in [8, 2048]; it is
    transformed in place and returned as the field."""
    import torch

    n = noise.shape[0]
    if noise.dim() != 3 or noise.shape != (n, n, n) or not noise.is_cuda:
        raise ValueError("noise must be a CUDA (N, N, N) tensor")
    dtype = {torch.float32: "f4", torch.float64: "f8"}.get(noise.dtype)
    if dtype is None:
        raise ValueError("noise must be float32 or float64")
    m = _lib.mesh_desc(n, boxsize, "cic", False, False, dtype)
    table = torch.from_numpy(amplitude_table(n, boxsize, pk)).to(noise.device)
    mesh = noise.contiguous()
    ctx.pk_fft_r2c(m, mesh)
    ctx.pk_shape_spectrum(m, mesh, table)
    ctx.pk_fft_c2r(m, mesh)
    return mesh
