"""Paper-vocabulary front end: ``to_mesh``, ``FFTPower`` and
``ConvolvedFFTPower`` (Sec. 3.3.2, 3.4.1).

These wrappers only turn keyword arguments into the C descriptors of
include/pk.h, allocate device buffers with PyTorch and call the library; the
estimator itself runs in the HIP kernels of libpk.

    mesh = to_mesh(pos, Nmesh=512, BoxSize=1380., resampler="tsc", interlaced=True)
    r = FFTPower(mesh, mode="2d", Nmu=5, poles=[0, 2, 4])
    r["k"], r["power"], r["modes"], r["poles"][2], r["power2d"], r["shotnoise"]
"""

import math

from . import _lib

_CONTEXTS = {}


def context(device=0):
    """The library context bound to ``device`` and torch's current stream there."""
    import torch

    stream = torch.cuda.current_stream(device)
    key = (device, stream.cuda_stream)
    ctx = _CONTEXTS.get(key)
    if ctx is None:
        ctx = _lib.Context(device, stream)
        _CONTEXTS[key] = ctx
    return ctx


class CatalogMesh:
    """A catalog bound to a mesh description (the paper's ``to_mesh`` result).

    ``pos`` is an (N_p, 3) tensor on the GPU in the precision of ``dtype``
    ('f4' or 'f8'); ``weight`` an optional (N_p,) tensor of the same dtype.
    """

    def __init__(self, pos, Nmesh, BoxSize, resampler="cic", interlaced=False,
                 compensated=True, dtype="f4", weight=None):
        import torch

        want = torch.float32 if dtype in ("f4", "float32") else torch.float64
        if pos.dtype != want or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_cuda:
            raise ValueError(f"pos must be a CUDA (N, 3) tensor of {want}")
        if weight is not None and (weight.dtype != want or weight.shape != (pos.shape[0],)
                                   or not weight.is_cuda or weight.device != pos.device):
            raise ValueError(f"weight must be an (N,) tensor of {want} on {pos.device}")
        self.pos = pos.contiguous()
        self.weight = None if weight is None else weight.contiguous()
        self.Nmesh = int(Nmesh)
        self.BoxSize = float(BoxSize)
        self.resampler = resampler
        self.interlaced = bool(interlaced)
        self.compensated = bool(compensated)
        self.dtype = "f4" if want == torch.float32 else "f8"
        self.desc = _lib.mesh_desc(self.Nmesh, self.BoxSize, resampler, interlaced,
                                   compensated, self.dtype)
        if _lib.mesh_bytes(self.desc) == 0:
            raise ValueError("invalid mesh description (Nmesh must be a power of two in [8, 2048])")

    @property
    def device(self):
        return self.pos.device.index or 0

    def paint(self, shift_cells=0.0):
        """The painted real mesh (N, N, N) of sum_p w_p W(u_p - j), Eq. (1)."""
        import torch

        n = self.Nmesh
        tdt = torch.float32 if self.dtype == "f4" else torch.float64
        mesh = torch.empty((n, n, n), dtype=tdt, device=self.pos.device)
        wsums = torch.empty(2, dtype=torch.float64, device=self.pos.device)
        context(self.device).pk_paint(self.desc, self.pos, self.weight, self.pos.shape[0],
                                      shift_cells, mesh, wsums)
        return mesh, wsums


def to_mesh(pos, Nmesh, BoxSize, resampler="cic", interlaced=False, compensated=True,
            dtype="f4", weight=None):
    return CatalogMesh(pos, Nmesh, BoxSize, resampler, interlaced, compensated, dtype, weight)


def bins_for(mesh, mode="1d", dk=None, kmin=0.0, kmax=None, Nmu=5, poles=(), los=(0, 0, 1)):
    """C bin descriptor from FFTPower keywords (k in units of h/Mpc, like L):
    bins of width dk (default k_f) from kmin, as many whole bins as fit below
    kmax (default the Nyquist wave number k_N = pi N / L)."""
    kf = 2.0 * math.pi / mesh.BoxSize
    dk_f = 1.0 if dk is None else float(dk) / kf
    kmin_f = float(kmin) / kf
    # whole bins whose top edge is at most kmax (default: the Nyquist index)
    kmax_f = mesh.Nmesh // 2 if kmax is None else float(kmax) / kf
    nk = _lib.num_kbins(kmin_f, dk_f, kmax_f)
    if nk == 0:
        raise ValueError("no whole k-bin of width dk fits between kmin and kmax")
    axis = [i for i, v in enumerate(los) if v][0]
    if sum(1 for v in los if v) != 1:
        raise ValueError("los must be a unit vector along one axis")
    nmu = int(Nmu) if mode == "2d" else 0
    return _lib.bin_desc(nk, kmin_f, dk_f, nmu, tuple(poles), axis)


def FFTPower(mesh, mode="1d", dk=None, kmin=0.0, kmax=None, Nmu=5, poles=(), los=(0, 0, 1),
             workspace=None):
    """Periodic-box power spectrum of a CatalogMesh (Sec. 3.4.1).

    Returns a dict with k, power, modes, poles {ell: P_ell}, and for
    mode='2d' k2d, mu2d, power2d, modes2d; plus shotnoise, wsum, w2sum.
    Shot noise is reported, not subtracted.
    """
    import torch

    b = bins_for(mesh, mode, dk, kmin, kmax, Nmu, poles, los)
    need = _lib.workspace_bytes(mesh.desc, b, mesh.pos.shape[0])
    if need == 0:
        raise ValueError("invalid binning for this mesh")
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=mesh.pos.device)
    result = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device=mesh.pos.device)
    ctx = context(mesh.device)
    ctx.pk_fftpower(mesh.desc, b, mesh.pos, mesh.weight, mesh.pos.shape[0], workspace, result)
    out = ctx.pk_result_to_host(mesh.desc, b, result)
    out["edges"] = (2 * math.pi / mesh.BoxSize) * (b.kmin_f + b.dk_f * __import__("numpy").arange(b.nk + 1))
    return out


def ConvolvedFFTPower(mesh, randoms, poles=(0, 2, 4), observer=(0.0, 0.0, 0.0), norm=None,
                      dk=None, kmin=0.0, kmax=None, randoms_weight=None, workspace=None):
    """Survey power multipoles with a varying line of sight (Sec. 3.4.1,
    ConvolvedFFTPower): ``mesh`` is the data CatalogMesh (window,
    compensation, precision; interlacing is not offered here), ``randoms`` a
    CUDA (N_r, 3) tensor of the same dtype and ``randoms_weight`` its optional
    weights.  ``observer`` is in box coordinates.  ``norm`` is the survey
    normalisation I of P_ell = (2 ell + 1) / I <Re F_0 F_ell*>; it depends on
    the survey's mean density, so it must be given.  Returns k, modes,
    poles {ell: P_ell}, shotnoise (reported, not subtracted), alpha, wsum,
    w2sum and the k edges."""
    import numpy as np
    import torch

    if norm is None:
        raise ValueError("norm (the survey normalisation I) must be given")
    if mesh.interlaced:
        raise ValueError("the survey multipoles are not offered for interlaced meshes")
    want = mesh.pos.dtype
    if (randoms.dtype != want or randoms.dim() != 2 or randoms.shape[1] != 3
            or not randoms.is_cuda):
        raise ValueError(f"randoms must be a CUDA (N, 3) tensor of {want}")
    if randoms.device != mesh.pos.device:
        raise ValueError(f"randoms must be on {mesh.pos.device}")
    if randoms_weight is not None and (randoms_weight.dtype != want
                                       or randoms_weight.shape != (randoms.shape[0],)
                                       or not randoms_weight.is_cuda
                                       or randoms_weight.device != randoms.device):
        raise ValueError(f"randoms_weight must be an (N,) tensor of {want} on {randoms.device}")
    b = bins_for(mesh, "1d", dk, kmin, kmax, 0, tuple(poles), (0, 0, 1))
    randoms = randoms.contiguous()
    nd, nr = mesh.pos.shape[0], randoms.shape[0]
    need = _lib.convolved_workspace_bytes(mesh.desc, b, nd, nr)
    if need == 0:
        raise ValueError("invalid binning or catalog sizes for the survey multipoles")
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=mesh.pos.device)
    result = torch.empty(_lib.convolved_doubles(b), dtype=torch.float64, device=mesh.pos.device)
    ctx = context(mesh.device)
    ctx.pk_convolved_power(mesh.desc, b, observer, mesh.pos, mesh.weight, nd, randoms,
                           None if randoms_weight is None else randoms_weight.contiguous(), nr,
                           workspace, result)
    out = ctx.pk_convolved_to_host(mesh.desc, b, norm, result)
    out["edges"] = (2 * math.pi / mesh.BoxSize) * (b.kmin_f + b.dk_f * np.arange(b.nk + 1))
    return out
