"""pkmi: the FFT power-spectrum hot path of nbodykit (Hand, Feng et al. 2018)
as a native MI355X (gfx950) library.

The compute path is the C-ABI library ``libpk.so`` built from ``csrc/``; the
Python layer only marshals arguments (``_lib``) and offers the paper's
vocabulary (``api.to_mesh`` / ``api.FFTPower``).  Importing this package does
not load the library; the first call that needs it does, and fails loudly if
it is missing.
"""

__version__ = "0.1.0"
