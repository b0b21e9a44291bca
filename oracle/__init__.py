"""FP64 CPU oracle for the FFT power-spectrum estimator (TEST INFRASTRUCTURE ONLY).

This package is the slow, plain reference that the GPU library is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does, and it imports nothing
from the GPU package.

What it computes follows the nbodykit paper (Hand, Feng et al. 2018):

* painting of F(x) = [1 + delta'(x)] V(x) with weights W   -- Sec. 3.3.1, Eq. (1)
* CIC / TSC / PCS mass-assignment windows, interlacing and
  window compensation                                      -- Sec. 3.3.2, Eq. (2)
* the periodic-box power estimator P(k), P(k, mu), P_ell(k) -- Sec. 3.4.1
* survey multipoles with a varying line of sight
  (ConvolvedFFTPower, named in Sec. 3.4.1)                 -- parity unpinned

Everything is evaluated in float64 with NumPy / SciPy; the only library
primitives used are ``np.floor``, ``np.bincount``, ``np.searchsorted`` and
``scipy.fft.rfftn``.

Pinning: every function here is checked by the ``-m "not gpu"`` tests against
closed forms, brute-force enumeration and exact identities.  The readings of
the paper that those tests pin are listed in the module docstrings.  One item
is "parity unpinned": the paper's own accuracy claims for interlaced windows
against a 2x-resolution reference (Sec. 3.3.2, discussion of Fig. 2) depend on
a mock that cannot be rebuilt, so they are context, not a pin.  The survey
multipoles are a second: the paper names that estimator without defining it,
so ``convolved`` follows its standard definition and is pinned against
identities, not against the paper.
"""

from .paint import (wrap_positions, cell_coordinates, window_weights, paint_mesh, paint_cells,
                    painted_modes)
from .power import (
    r2c,
    c2r,
    mode_indices,
    interlace_combine,
    compensate,
    kbin_edges_sq,
    kbin_index,
    mubin_index,
    legendre,
    fftpower_from_spectra,
    fftpower,
    mode_tables,
    prepared_spectrum,
    cross_from_spectra,
    projected_power,
)
from .convolved import real_ylm, unit_vectors, k_unit_vectors, multipole_fields, convolved_power

__all__ = [
    "wrap_positions",
    "cell_coordinates",
    "window_weights",
    "paint_mesh",
    "paint_cells",
    "painted_modes",
    "r2c",
    "c2r",
    "mode_indices",
    "interlace_combine",
    "compensate",
    "kbin_edges_sq",
    "kbin_index",
    "mubin_index",
    "legendre",
    "fftpower_from_spectra",
    "fftpower",
    "mode_tables",
    "prepared_spectrum",
    "cross_from_spectra",
    "projected_power",
    "real_ylm",
    "unit_vectors",
    "k_unit_vectors",
    "multipole_fields",
    "convolved_power",
]
