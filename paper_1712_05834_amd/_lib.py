"""ctypes binding of libpk (include/pk.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all
arithmetic of the hot path runs in the HIP kernels of ``libpk.so``.  Device
buffers are passed as torch tensors (their ``data_ptr()``), streams as the
HIP stream handle of the current torch stream.  If the library is missing the
first call raises: there is no CPU fallback.
"""

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PK_LIBRARY", os.path.join(HERE, "libpk.so"))

PK_OK, PK_EINVAL, PK_ENOMEM, PK_EDEVICE, PK_EUNSUPPORTED = 0, -1, -2, -3, -4
PK_F32, PK_F64 = 0, 1
WINDOWS = {"cic": 2, "tsc": 3, "pcs": 4}

# Every symbol include/pk.h declares.
EXPORTS = (
    "pk_ctx_create", "pk_ctx_destroy", "pk_last_error", "pk_mesh_bytes",
    "pk_result_doubles", "pk_workspace_bytes", "pk_ctx_table_bytes", "pk_paint",
    "pk_fft_r2c", "pk_compensate", "pk_bin_power", "pk_fftpower", "pk_result_to_host",
    "pk_ctx_set_timing", "pk_stage_count", "pk_stage_name", "pk_ctx_stage_times",
    "pk_ctx_set_lanes", "pk_ctx_lanes", "pk_fftpower_async", "pk_lane_query", "pk_lane_wait",
    "pk_fftpower_batch", "pk_bin_cross", "pk_fftpower_v", "pk_projected_doubles",
    "pk_bin_projected", "pk_projected_to_host", "pk_convolved_doubles",
    "pk_convolved_workspace_bytes", "pk_convolved_power", "pk_convolved_to_host", "pk_fft_c2r",
    "pk_shape_table_len", "pk_shape_spectrum", "pk_num_kbins", "pk_bin_power_noalloc",
    "pk_fftpower_batch_graph", "pk_graph_launch", "pk_graph_nodes", "pk_graph_destroy",
    "pk_ctx_set_autotune", "pk_tune_count", "pk_tune_get", "pk_tune_put",
)
PK_MAX_LANES = 64
PK_DEVICE_NONE = -1


class PkError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libpk status {status}: {message}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("nmesh", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("interlaced", ctypes.c_int32),
        ("compensated", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("boxsize", ctypes.c_double),
    ]


class BinDesc(ctypes.Structure):
    _fields_ = [
        ("kmin_f", ctypes.c_double),
        ("dk_f", ctypes.c_double),
        ("nk", ctypes.c_int32),
        ("nmu", ctypes.c_int32),
        ("npoles", ctypes.c_int32),
        ("poles", ctypes.c_int32 * 4),
        ("los", ctypes.c_int32),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("nmesh", ctypes.c_int32), ("dtype", ctypes.c_int32), ("window", ctypes.c_int32),
        ("interlaced", ctypes.c_int32), ("density", ctypes.c_int32), ("split", ctypes.c_int32),
        ("xpass_per_cu", ctypes.c_int32), ("ms", ctypes.c_double),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.POINTER(ctypes.c_double)),
        ("power", ctypes.POINTER(ctypes.c_double)),
        ("modes", ctypes.POINTER(ctypes.c_int64)),
        ("poles", ctypes.POINTER(ctypes.c_double)),
        ("k2d", ctypes.POINTER(ctypes.c_double)),
        ("mu2d", ctypes.POINTER(ctypes.c_double)),
        ("power2d", ctypes.POINTER(ctypes.c_double)),
        ("modes2d", ctypes.POINTER(ctypes.c_int64)),
        ("shotnoise", ctypes.c_double),
        ("wsum", ctypes.c_double),
        ("w2sum", ctypes.c_double),
    ]


_lib = None
_lock = threading.Lock()


def load(path=None):
    """Loads libpk.so once (raises if it is missing or incomplete)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(
                f"{p} is missing: build it with `python -m paper_1712_05834_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(p)
        for name in EXPORTS:
            getattr(lib, name)  # AttributeError if the symbol is absent
        vp, i32, i64, sz, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_size_t, ctypes.c_double)
        md, bd = ctypes.POINTER(MeshDesc), ctypes.POINTER(BinDesc)
        sig = {
            "pk_ctx_create": (i32, [ctypes.POINTER(vp), ctypes.c_int, vp]),
            "pk_ctx_destroy": (None, [vp]),
            "pk_last_error": (ctypes.c_char_p, [vp]),
            "pk_mesh_bytes": (sz, [md]),
            "pk_result_doubles": (sz, [bd]),
            "pk_num_kbins": (i32, [dbl, dbl, dbl]),
            "pk_workspace_bytes": (sz, [md, bd, i64]),
            "pk_ctx_table_bytes": (sz, [vp]),
            "pk_paint": (i32, [vp, md, vp, vp, i64, dbl, vp, vp]),
            "pk_fft_r2c": (i32, [vp, md, vp]),
            "pk_fft_c2r": (i32, [vp, md, vp]),
            "pk_shape_table_len": (i64, [md]),
            "pk_shape_spectrum": (i32, [vp, md, vp, vp, i64]),
            "pk_compensate": (i32, [vp, md, vp, vp]),
            "pk_bin_power": (i32, [vp, md, bd, vp, vp]),
            "pk_bin_power_noalloc": (i32, [vp, md, bd, vp, vp]),
            "pk_bin_cross": (i32, [vp, md, bd, vp, vp, vp]),
            "pk_projected_doubles": (sz, [bd]),
            "pk_bin_projected": (i32, [vp, md, bd, ctypes.c_int, vp, vp]),
            "pk_projected_to_host": (i32, [vp, md, bd, ctypes.c_int, vp,
                                           ctypes.POINTER(Result)]),
            "pk_fftpower": (i32, [vp, md, bd, vp, vp, i64, vp, sz, vp]),
            "pk_fftpower_v": (i32, [vp, md, bd, vp, vp, vp, i64, vp, sz, vp]),
            "pk_result_to_host": (i32, [vp, md, bd, vp, ctypes.POINTER(Result)]),
            "pk_ctx_set_timing": (i32, [vp, ctypes.c_int]),
            "pk_stage_count": (ctypes.c_int, []),
            "pk_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
            "pk_ctx_stage_times": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
            "pk_ctx_set_lanes": (i32, [vp, ctypes.c_int]),
            "pk_ctx_lanes": (ctypes.c_int, [vp]),
            "pk_fftpower_async": (i32, [vp, ctypes.c_int, md, bd, vp, vp, i64, vp, sz, vp]),
            "pk_lane_query": (ctypes.c_int, [vp, ctypes.c_int]),
            "pk_lane_wait": (i32, [vp, ctypes.c_int]),
            "pk_fftpower_batch": (i32, [vp, ctypes.c_int, md, bd, ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.POINTER(i64),
                                        ctypes.POINTER(vp), sz, ctypes.POINTER(vp)]),
            "pk_fftpower_batch_graph": (i32, [vp, ctypes.c_int, md, bd, ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(i64),
                                              ctypes.POINTER(vp), sz, ctypes.POINTER(vp),
                                              ctypes.POINTER(vp)]),
            "pk_graph_launch": (i32, [vp, vp]),
            "pk_ctx_set_autotune": (i32, [vp, ctypes.c_int]),
            "pk_tune_count": (ctypes.c_int, [vp]),
            "pk_tune_get": (i32, [vp, ctypes.c_int, ctypes.POINTER(TuneEntry)]),
            "pk_tune_put": (i32, [vp, ctypes.POINTER(TuneEntry)]),
            "pk_graph_nodes": (sz, [vp]),
            "pk_graph_destroy": (None, [vp]),
            "pk_convolved_doubles": (sz, [bd]),
            "pk_convolved_workspace_bytes": (sz, [md, bd, i64, i64]),
            "pk_convolved_power": (i32, [vp, md, bd, ctypes.POINTER(dbl), vp, vp, i64, vp, vp,
                                         i64, vp, sz, vp]),
            "pk_convolved_to_host": (i32, [vp, md, bd, dbl, vp, ctypes.POINTER(Result)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def mesh_desc(nmesh, boxsize, window="cic", interlaced=False, compensated=True, dtype="f4"):
    w = WINDOWS[window] if isinstance(window, str) else int(window)
    dt = {"f4": PK_F32, "f8": PK_F64, "float32": PK_F32, "float64": PK_F64}[str(dtype)]
    return MeshDesc(int(nmesh), w, int(bool(interlaced)), int(bool(compensated)), dt, 0,
                    float(boxsize))


def bin_desc(nk, kmin_f=0.0, dk_f=1.0, nmu=0, poles=(), los=2):
    poles = tuple(int(p) for p in poles)
    arr = (ctypes.c_int32 * 4)(*(list(poles) + [0] * (4 - len(poles)))[:4])
    return BinDesc(float(kmin_f), float(dk_f), int(nk), int(nmu), len(poles), arr, int(los))


def num_kbins(kmin_f, dk_f, kmax_f):
    """pk_num_kbins: whole k-bins of width dk_f from kmin_f whose top edge is
    at most kmax_f (units of k_f).  Raises ValueError for invalid edges."""
    nk = int(load().pk_num_kbins(float(kmin_f), float(dk_f), float(kmax_f)))
    if nk < 0:
        raise ValueError(f"invalid k-bin edges kmin={kmin_f}, dk={dk_f}, kmax={kmax_f} "
                         f"(status {nk})")
    return nk


def mesh_bytes(m):
    return int(load().pk_mesh_bytes(ctypes.byref(m)))


def result_doubles(b):
    return int(load().pk_result_doubles(ctypes.byref(b)))


def projected_doubles(b):
    return int(load().pk_projected_doubles(ctypes.byref(b)))


def shape_table_len(m):
    return int(load().pk_shape_table_len(ctypes.byref(m)))


def convolved_doubles(b):
    return int(load().pk_convolved_doubles(ctypes.byref(b)))


def convolved_workspace_bytes(m, b, n_data, n_rand):
    return int(load().pk_convolved_workspace_bytes(ctypes.byref(m), ctypes.byref(b),
                                                   int(n_data), int(n_rand)))


def workspace_bytes(m, b, npart):
    return int(load().pk_workspace_bytes(ctypes.byref(m), ctypes.byref(b), int(npart)))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def mesh_torch_dtype(m):
    """torch dtype of positions, weights and meshes of a mesh description."""
    import torch

    return torch.float32 if m.dtype == PK_F32 else torch.float64


def device_arg(t, name, device, dtype=None, numel=0, nbytes=0, optional=False):
    """Checks a tensor before its address crosses the C ABI, and returns that
    address: a contiguous tensor on GPU ``device`` (any GPU for a
    validation-only context, device < 0), of ``dtype`` when given, with at
    least ``numel`` elements and ``nbytes`` bytes.  The library reads raw
    addresses, so a host tensor or a short buffer would be a device memory
    fault; here it is a ValueError before any launch."""
    import torch

    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, not {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (got a tensor on {t.device})")
    if device is not None and device >= 0 and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} are needed")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, {nbytes} are "
                         "needed")
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """A captured batch (pk_fftpower_batch_graph): launch() replays it on the
    context's stream.  It holds references to the arrays it was built with."""

    def __init__(self, ctx, handle, keep):
        self.ctx, self.handle, self._keep = ctx, handle, keep

    @property
    def nodes(self):
        return int(self.ctx.lib.pk_graph_nodes(self.handle))

    def launch(self):
        self.ctx._check(self.ctx.lib.pk_graph_launch(self.ctx.handle, self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.pk_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One pk_ctx bound to a device and a HIP stream.

    ``device=PK_DEVICE_NONE`` (-1) gives a validation-only context: every
    argument is checked as on a device, and calls that would reach a device
    fail with PK_EDEVICE (no GPU needed).  Every tensor argument is checked by
    ``device_arg`` before its address is passed to the library."""

    def __init__(self, device=0, stream=None):
        self.lib = load()
        handle = ctypes.c_void_p()
        if device == PK_DEVICE_NONE:
            self.stream = None
            st = self.lib.pk_ctx_create(ctypes.byref(handle), PK_DEVICE_NONE, None)
        else:
            import torch

            if stream is None:
                stream = torch.cuda.current_stream(device)
            self.stream = stream
            st = self.lib.pk_ctx_create(ctypes.byref(handle), int(device),
                                        ctypes.c_void_p(stream.cuda_stream))
        if st != PK_OK:
            raise PkError(st, self.lib.pk_last_error(None).decode())
        self.handle = handle
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pk_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PK_OK:
            raise PkError(st, self.lib.pk_last_error(self.handle).decode())

    # ---- argument checks (shapes from the descriptors; nothing is launched)

    def _arg(self, t, name, **kw):
        return device_arg(t, name, self.device, **kw)

    def _mesh_arg(self, m, t, name, optional=False):
        """A real mesh or packed spectrum of m: the mesh dtype, pk_mesh_bytes."""
        return self._arg(t, name, dtype=mesh_torch_dtype(m), nbytes=mesh_bytes(m),
                         optional=optional)

    def _catalog_args(self, m, pos, weight, n, names=("pos", "weight")):
        n = int(n)
        dt = mesh_torch_dtype(m)
        return (self._arg(pos, names[0], dtype=dt, numel=3 * n, optional=n == 0),
                self._arg(weight, names[1], dtype=dt, numel=n, optional=True))

    def _f64_arg(self, t, name, count, optional=False):
        import torch

        return self._arg(t, name, dtype=torch.float64, numel=count, optional=optional)

    def _result_arg(self, b, t):
        return self._f64_arg(t, "result", result_doubles(b))

    @staticmethod
    def _nbytes(t):
        return 0 if t is None else t.numel() * t.element_size()

    # ---- run-time tuning

    def pk_ctx_set_autotune(self, mode):
        self._check(self.lib.pk_ctx_set_autotune(self.handle, int(mode)))

    def tune_table(self):
        """The tuned launch choices as a list of dicts (to be stored)."""
        out = []
        for i in range(int(self.lib.pk_tune_count(self.handle))):
            e = TuneEntry()
            self._check(self.lib.pk_tune_get(self.handle, i, ctypes.byref(e)))
            out.append({f: getattr(e, f) for f, _ in TuneEntry._fields_})
        return out

    def tune_load(self, table):
        """Loads entries of tune_table() (from this or another context)."""
        for d in table:
            e = TuneEntry(*[d[f] for f, _ in TuneEntry._fields_])
            self._check(self.lib.pk_tune_put(self.handle, ctypes.byref(e)))

    # ---- diagnostics

    def pk_ctx_set_timing(self, enable):
        self._check(self.lib.pk_ctx_set_timing(self.handle, int(bool(enable))))

    def stage_names(self):
        return [self.lib.pk_stage_name(i).decode() for i in range(self.lib.pk_stage_count())]

    def pk_ctx_stage_times(self):
        n = self.lib.pk_stage_count()
        arr = (ctypes.c_double * n)()
        self._check(self.lib.pk_ctx_stage_times(self.handle, arr))
        return dict(zip(self.stage_names(), list(arr)))

    def table_bytes(self):
        return int(self.lib.pk_ctx_table_bytes(self.handle))

    # ---- stages

    def pk_paint(self, m, pos, weight, n, shift_cells, mesh, wsums=None):
        p, w = self._catalog_args(m, pos, weight, n)
        mp = self._mesh_arg(m, mesh, "mesh")
        ws = self._f64_arg(wsums, "wsums", 2, optional=True)
        self._check(self.lib.pk_paint(self.handle, ctypes.byref(m), p, w, int(n),
                                      float(shift_cells), mp, ws))

    def pk_fft_r2c(self, m, mesh):
        self._check(self.lib.pk_fft_r2c(self.handle, ctypes.byref(m),
                                        self._mesh_arg(m, mesh, "mesh")))

    def pk_fft_c2r(self, m, mesh):
        self._check(self.lib.pk_fft_c2r(self.handle, ctypes.byref(m),
                                        self._mesh_arg(m, mesh, "mesh")))

    def pk_shape_spectrum(self, m, cmesh, table):
        c = self._mesh_arg(m, cmesh, "cmesh")
        tb = self._f64_arg(table, "table", shape_table_len(m))
        self._check(self.lib.pk_shape_spectrum(self.handle, ctypes.byref(m), c, tb,
                                               int(table.numel())))

    def pk_compensate(self, m, cmesh, cmesh_b=None):
        c = self._mesh_arg(m, cmesh, "cmesh")
        cb = self._mesh_arg(m, cmesh_b, "cmesh_b", optional=True)
        self._check(self.lib.pk_compensate(self.handle, ctypes.byref(m), c, cb))

    def pk_bin_power(self, m, b, cmesh, result):
        c = self._mesh_arg(m, cmesh, "cmesh")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_bin_power(self.handle, ctypes.byref(m), ctypes.byref(b), c, r))

    def pk_bin_power_noalloc(self, m, b, cmesh, result):
        c = self._mesh_arg(m, cmesh, "cmesh")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_bin_power_noalloc(self.handle, ctypes.byref(m), ctypes.byref(b),
                                                  c, r))

    def pk_bin_cross(self, m, b, cmesh1, cmesh2, result):
        c1 = self._mesh_arg(m, cmesh1, "cmesh1")
        c2 = self._mesh_arg(m, cmesh2, "cmesh2")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_bin_cross(self.handle, ctypes.byref(m), ctypes.byref(b),
                                          c1, c2, r))

    def pk_bin_projected(self, m, b, keep, cmesh, result):
        c = self._mesh_arg(m, cmesh, "cmesh")
        r = self._f64_arg(result, "result", projected_doubles(b))
        self._check(self.lib.pk_bin_projected(self.handle, ctypes.byref(m), ctypes.byref(b),
                                              int(keep), c, r))

    def pk_projected_to_host(self, m, b, keep, result):
        import numpy as np

        rp = self._f64_arg(result, "result", projected_doubles(b))
        nk = b.nk
        out = {"k": np.empty(nk), "power": np.empty(nk), "modes": np.empty(nk, dtype=np.int64)}
        dbl, i64 = ctypes.c_double, ctypes.c_int64
        r = Result(out["k"].ctypes.data_as(ctypes.POINTER(dbl)),
                   out["power"].ctypes.data_as(ctypes.POINTER(dbl)),
                   out["modes"].ctypes.data_as(ctypes.POINTER(i64)),
                   None, None, None, None, None, 0.0, 0.0, 0.0)
        self._check(self.lib.pk_projected_to_host(self.handle, ctypes.byref(m), ctypes.byref(b),
                                                  int(keep), rp, ctypes.byref(r)))
        out["poles"] = {}
        out["shotnoise"], out["wsum"], out["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        return out

    def pk_convolved_power(self, m, b, observer, data_pos, data_weight, n_data, rand_pos,
                           rand_weight, n_rand, workspace, result):
        dp, dw = self._catalog_args(m, data_pos, data_weight, n_data,
                                    ("data_pos", "data_weight"))
        rp, rw = self._catalog_args(m, rand_pos, rand_weight, n_rand,
                                    ("rand_pos", "rand_weight"))
        ws = self._arg(workspace, "workspace")
        res = self._f64_arg(result, "result", convolved_doubles(b))
        obs = (ctypes.c_double * 3)(*[float(v) for v in observer])
        self._check(self.lib.pk_convolved_power(
            self.handle, ctypes.byref(m), ctypes.byref(b), obs, dp, dw, int(n_data), rp, rw,
            int(n_rand), ws, self._nbytes(workspace), res))

    def pk_convolved_to_host(self, m, b, norm, result):
        """Host dict: k, modes, poles {ell: P_ell}, shotnoise, wsum / w2sum of
        the data, and alpha read from the weight sums of the result."""
        import numpy as np

        rp = self._f64_arg(result, "result", convolved_doubles(b))
        nk = b.nk
        out = {"k": np.empty(nk), "modes": np.empty(nk, dtype=np.int64)}
        poles = np.empty((b.npoles, nk))
        dbl, i64 = ctypes.c_double, ctypes.c_int64
        r = Result(out["k"].ctypes.data_as(ctypes.POINTER(dbl)), None,
                   out["modes"].ctypes.data_as(ctypes.POINTER(i64)),
                   poles.ctypes.data_as(ctypes.POINTER(dbl)), None, None, None, None,
                   0.0, 0.0, 0.0)
        self._check(self.lib.pk_convolved_to_host(self.handle, ctypes.byref(m), ctypes.byref(b),
                                                  float(norm), rp, ctypes.byref(r)))
        out["poles"] = {int(b.poles[i]): poles[i] for i in range(b.npoles)}
        out["shotnoise"], out["wsum"], out["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        sums = result[b.npoles * nk:b.npoles * nk + 4].double().cpu().numpy()
        out["alpha"] = float(sums[0] / sums[2])
        return out

    def pk_fftpower(self, m, b, pos, weight, n, workspace, result):
        p, w = self._catalog_args(m, pos, weight, n)
        ws = self._arg(workspace, "workspace")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_fftpower(self.handle, ctypes.byref(m), ctypes.byref(b), p, w,
                                         int(n), ws, self._nbytes(workspace), r))

    def pk_fftpower_v(self, m, b, pos, weight, value, n, workspace, result):
        p, w = self._catalog_args(m, pos, weight, n)
        v = self._arg(value, "value", dtype=mesh_torch_dtype(m), numel=int(n), optional=True)
        ws = self._arg(workspace, "workspace")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_fftpower_v(self.handle, ctypes.byref(m), ctypes.byref(b), p, w,
                                           v, int(n), ws, self._nbytes(workspace), r))

    # ---- lanes

    def pk_ctx_set_lanes(self, nlanes):
        self._check(self.lib.pk_ctx_set_lanes(self.handle, int(nlanes)))

    def pk_ctx_lanes(self):
        return int(self.lib.pk_ctx_lanes(self.handle))

    def pk_fftpower_async(self, lane, m, b, pos, weight, n, workspace, result):
        p, w = self._catalog_args(m, pos, weight, n)
        ws = self._arg(workspace, "workspace")
        r = self._result_arg(b, result)
        self._check(self.lib.pk_fftpower_async(self.handle, int(lane), ctypes.byref(m),
                                               ctypes.byref(b), p, w, int(n), ws,
                                               self._nbytes(workspace), r))

    def pk_lane_query(self, lane):
        st = int(self.lib.pk_lane_query(self.handle, int(lane)))
        if st < 0:
            self._check(st)
        return st == 1

    def pk_lane_wait(self, lane):
        self._check(self.lib.pk_lane_wait(self.handle, int(lane)))

    def pk_fftpower_batch(self, ms, bs, pos, weights, ns, lane_workspaces, results):
        """ms, bs: sequences of MeshDesc / BinDesc; pos, weights (None entries
        allowed), results: sequences of device tensors; lane_workspaces: one
        device tensor per lane, all of the same size."""
        self._check(self.lib.pk_fftpower_batch(
            self.handle, *self._batch_args(ms, bs, pos, weights, ns, lane_workspaces, results)))

    def pk_fftpower_batch_graph(self, ms, bs, pos, weights, ns, lane_workspaces, results):
        """The batch captured into a HIP graph (pk_fftpower_batch_graph); the
        returned Graph replays it with launch().  Every tensor passed must
        stay alive while the graph is used."""
        g = ctypes.c_void_p()
        args = self._batch_args(ms, bs, pos, weights, ns, lane_workspaces, results,
                                need_lanes=False)
        self._check(self.lib.pk_fftpower_batch_graph(self.handle, *args, ctypes.byref(g)))
        return Graph(self, g, keep=(args, list(pos), list(weights), list(lane_workspaces),
                                    list(results)))

    def _batch_args(self, ms, bs, pos, weights, ns, lane_workspaces, results, need_lanes=True):
        count = len(ms)
        if not (len(bs) == len(pos) == len(weights) == len(ns) == len(results) == count):
            raise ValueError("batch arguments must all have one entry per request")
        vp = ctypes.c_void_p
        pp, wp, rp = [], [], []
        for i in range(count):
            p, w = self._catalog_args(ms[i], pos[i], weights[i], ns[i],
                                      (f"pos[{i}]", f"weight[{i}]"))
            pp.append(p)
            wp.append(w)
            rp.append(self._f64_arg(results[i], f"result[{i}]", result_doubles(bs[i])))
        if not lane_workspaces:
            raise ValueError("one workspace per lane is needed")
        nbytes = self._nbytes(lane_workspaces[0])
        lw = [self._arg(t, f"lane_workspace[{j}]", nbytes=nbytes)
              for j, t in enumerate(lane_workspaces)]
        if any(self._nbytes(t) != nbytes for t in lane_workspaces):
            raise ValueError("every lane workspace must have the same size")
        marr = (MeshDesc * max(count, 1))(*ms)
        barr = (BinDesc * max(count, 1))(*bs)

        def arr(ptrs):
            return (vp * max(len(ptrs), 1))(*[None if q is None else q.value for q in ptrs])

        narr = (ctypes.c_int64 * max(count, 1))(*[int(n) for n in ns])
        return (count, marr, barr, arr(pp), arr(wp), narr, arr(lw), nbytes, arr(rp))

    # ---- finalisation

    def pk_result_to_host(self, m, b, result):
        import numpy as np

        rp = self._result_arg(b, result)
        nk, nmu, npoles = b.nk, b.nmu, b.npoles
        out = {
            "k": np.empty(nk), "power": np.empty(nk), "modes": np.empty(nk, dtype=np.int64),
            "poles": np.empty((max(npoles, 1), nk)),
        }
        two = nmu > 1
        if two:
            for key in ("k2d", "mu2d", "power2d"):
                out[key] = np.empty((nk, nmu))
            out["modes2d"] = np.empty((nk, nmu), dtype=np.int64)

        def p(a, ct):
            return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None

        dbl, i64 = ctypes.c_double, ctypes.c_int64
        r = Result(p(out["k"], dbl), p(out["power"], dbl), p(out["modes"], i64),
                   p(out["poles"], dbl), p(out.get("k2d"), dbl), p(out.get("mu2d"), dbl),
                   p(out.get("power2d"), dbl), p(out.get("modes2d"), i64), 0.0, 0.0, 0.0)
        self._check(self.lib.pk_result_to_host(self.handle, ctypes.byref(m), ctypes.byref(b),
                                               rp, ctypes.byref(r)))
        res = {k: v for k, v in out.items() if k != "poles"}
        res["poles"] = {int(b.poles[i]): out["poles"][i].copy() for i in range(npoles)}
        res["shotnoise"], res["wsum"], res["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        return res
