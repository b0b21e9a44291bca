"""Host-side conversion between the library's packed half spectrum and the
(N, N, N/2 + 1) r2c array of the oracle (test glue: layout only).

Packed element kz' = 0 holds Z = c(kx, ky, 0) + i c(kx, ky, N/2); the other
columns are c(kx, ky, kz') unchanged.
"""

import numpy as np


def pack(c):
    n = c.shape[0]
    out = np.empty((n, n, n // 2), dtype=np.complex128)
    out[:, :, 1:] = c[:, :, 1 : n // 2]
    out[:, :, 0] = c[:, :, 0] + 1j * c[:, :, n // 2]
    return out


def unpack(z):
    n = z.shape[0]
    out = np.empty((n, n, n // 2 + 1), dtype=np.complex128)
    out[:, :, 1 : n // 2] = z[:, :, 1:]
    zz = z[:, :, 0]
    neg = (-np.arange(n)) % n
    zp = np.conj(zz[neg][:, neg])
    out[:, :, 0] = 0.5 * (zz + zp)
    out[:, :, n // 2] = (zz - zp) / 2j
    return out


def as_complex(t):
    """Device/host real array of N^3 values viewed as packed complex (N, N, N/2)."""
    a = np.asarray(t)
    n = a.shape[0]
    return a.reshape(n, n, n // 2, 2)[..., 0] + 1j * a.reshape(n, n, n // 2, 2)[..., 1]


def to_real_view(z, dtype):
    n = z.shape[0]
    out = np.empty((n, n, n // 2, 2), dtype=dtype)
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return out.reshape(n, n, n)
