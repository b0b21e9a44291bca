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
    "pk_shape_table_len", "pk_shape_spectrum",
)
PK_MAX_LANES = 64


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
            "pk_workspace_bytes": (sz, [md, bd, i64]),
            "pk_ctx_table_bytes": (sz, [vp]),
            "pk_paint": (i32, [vp, md, vp, vp, i64, dbl, vp, vp]),
            "pk_fft_r2c": (i32, [vp, md, vp]),
            "pk_fft_c2r": (i32, [vp, md, vp]),
            "pk_shape_table_len": (i64, [md]),
            "pk_shape_spectrum": (i32, [vp, md, vp, vp, i64]),
            "pk_compensate": (i32, [vp, md, vp, vp]),
            "pk_bin_power": (i32, [vp, md, bd, vp, vp]),
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


class Context:
    """One pk_ctx bound to a device and a HIP stream."""

    def __init__(self, device=0, stream=None):
        import torch

        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        handle = ctypes.c_void_p()
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

    def pk_paint(self, m, pos, weight, n, shift_cells, mesh, wsums=None):
        self._check(self.lib.pk_paint(self.handle, ctypes.byref(m), _ptr(pos), _ptr(weight),
                                      int(n), float(shift_cells), _ptr(mesh), _ptr(wsums)))

    def pk_fft_r2c(self, m, mesh):
        self._check(self.lib.pk_fft_r2c(self.handle, ctypes.byref(m), _ptr(mesh)))

    def pk_fft_c2r(self, m, mesh):
        self._check(self.lib.pk_fft_c2r(self.handle, ctypes.byref(m), _ptr(mesh)))

    def pk_shape_spectrum(self, m, cmesh, table):
        self._check(self.lib.pk_shape_spectrum(self.handle, ctypes.byref(m), _ptr(cmesh),
                                               _ptr(table), int(table.numel())))

    def pk_compensate(self, m, cmesh, cmesh_b=None):
        self._check(self.lib.pk_compensate(self.handle, ctypes.byref(m), _ptr(cmesh),
                                           _ptr(cmesh_b)))

    def pk_bin_power(self, m, b, cmesh, result):
        self._check(self.lib.pk_bin_power(self.handle, ctypes.byref(m), ctypes.byref(b),
                                          _ptr(cmesh), _ptr(result)))

    def pk_bin_cross(self, m, b, cmesh1, cmesh2, result):
        self._check(self.lib.pk_bin_cross(self.handle, ctypes.byref(m), ctypes.byref(b),
                                          _ptr(cmesh1), _ptr(cmesh2), _ptr(result)))

    def pk_bin_projected(self, m, b, keep, cmesh, result):
        self._check(self.lib.pk_bin_projected(self.handle, ctypes.byref(m), ctypes.byref(b),
                                              int(keep), _ptr(cmesh), _ptr(result)))

    def pk_projected_to_host(self, m, b, keep, result):
        import numpy as np

        nk = b.nk
        out = {"k": np.empty(nk), "power": np.empty(nk), "modes": np.empty(nk, dtype=np.int64)}
        dbl, i64 = ctypes.c_double, ctypes.c_int64
        r = Result(out["k"].ctypes.data_as(ctypes.POINTER(dbl)),
                   out["power"].ctypes.data_as(ctypes.POINTER(dbl)),
                   out["modes"].ctypes.data_as(ctypes.POINTER(i64)),
                   None, None, None, None, None, 0.0, 0.0, 0.0)
        self._check(self.lib.pk_projected_to_host(self.handle, ctypes.byref(m), ctypes.byref(b),
                                                  int(keep), _ptr(result), ctypes.byref(r)))
        out["poles"] = {}
        out["shotnoise"], out["wsum"], out["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        return out

    def pk_convolved_power(self, m, b, observer, data_pos, data_weight, n_data, rand_pos,
                           rand_weight, n_rand, workspace, result):
        nbytes = workspace.numel() * workspace.element_size()
        obs = (ctypes.c_double * 3)(*[float(v) for v in observer])
        self._check(self.lib.pk_convolved_power(
            self.handle, ctypes.byref(m), ctypes.byref(b), obs, _ptr(data_pos),
            _ptr(data_weight), int(n_data), _ptr(rand_pos), _ptr(rand_weight), int(n_rand),
            _ptr(workspace), nbytes, _ptr(result)))

    def pk_convolved_to_host(self, m, b, norm, result):
        """Host dict: k, modes, poles {ell: P_ell}, shotnoise, wsum / w2sum of
        the data, and alpha read from the weight sums of the result."""
        import numpy as np

        nk = b.nk
        out = {"k": np.empty(nk), "modes": np.empty(nk, dtype=np.int64)}
        poles = np.empty((b.npoles, nk))
        dbl, i64 = ctypes.c_double, ctypes.c_int64
        r = Result(out["k"].ctypes.data_as(ctypes.POINTER(dbl)), None,
                   out["modes"].ctypes.data_as(ctypes.POINTER(i64)),
                   poles.ctypes.data_as(ctypes.POINTER(dbl)), None, None, None, None,
                   0.0, 0.0, 0.0)
        self._check(self.lib.pk_convolved_to_host(self.handle, ctypes.byref(m), ctypes.byref(b),
                                                  float(norm), _ptr(result), ctypes.byref(r)))
        out["poles"] = {int(b.poles[i]): poles[i] for i in range(b.npoles)}
        out["shotnoise"], out["wsum"], out["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        sums = result[b.npoles * nk:b.npoles * nk + 4].double().cpu().numpy()
        out["alpha"] = float(sums[0] / sums[2])
        return out

    def pk_fftpower(self, m, b, pos, weight, n, workspace, result):
        nbytes = workspace.numel() * workspace.element_size()
        self._check(self.lib.pk_fftpower(self.handle, ctypes.byref(m), ctypes.byref(b), _ptr(pos),
                                         _ptr(weight), int(n), _ptr(workspace), nbytes,
                                         _ptr(result)))

    def pk_fftpower_v(self, m, b, pos, weight, value, n, workspace, result):
        nbytes = workspace.numel() * workspace.element_size()
        self._check(self.lib.pk_fftpower_v(self.handle, ctypes.byref(m), ctypes.byref(b),
                                           _ptr(pos), _ptr(weight), _ptr(value), int(n),
                                           _ptr(workspace), nbytes, _ptr(result)))

    def pk_ctx_set_lanes(self, nlanes):
        self._check(self.lib.pk_ctx_set_lanes(self.handle, int(nlanes)))

    def pk_ctx_lanes(self):
        return int(self.lib.pk_ctx_lanes(self.handle))

    def pk_fftpower_async(self, lane, m, b, pos, weight, n, workspace, result):
        nbytes = workspace.numel() * workspace.element_size()
        self._check(self.lib.pk_fftpower_async(self.handle, int(lane), ctypes.byref(m),
                                               ctypes.byref(b), _ptr(pos), _ptr(weight), int(n),
                                               _ptr(workspace), nbytes, _ptr(result)))

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
        count = len(ms)
        marr = (MeshDesc * max(count, 1))(*ms)
        barr = (BinDesc * max(count, 1))(*bs)
        vp = ctypes.c_void_p

        def ptrs(ts):
            return (vp * max(len(ts), 1))(*[None if t is None else t.data_ptr() for t in ts])

        nbytes = lane_workspaces[0].numel() * lane_workspaces[0].element_size()
        assert all(w.numel() * w.element_size() == nbytes for w in lane_workspaces)
        narr = (ctypes.c_int64 * max(count, 1))(*[int(n) for n in ns])
        self._check(self.lib.pk_fftpower_batch(
            self.handle, count, marr, barr, ptrs(pos), ptrs(weights), narr,
            ptrs(lane_workspaces), nbytes, ptrs(results)))

    def pk_result_to_host(self, m, b, result):
        import numpy as np

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
                                               _ptr(result), ctypes.byref(r)))
        res = {k: v for k, v in out.items() if k != "poles"}
        res["poles"] = {int(b.poles[i]): out["poles"][i].copy() for i in range(npoles)}
        res["shotnoise"], res["wsum"], res["w2sum"] = r.shotnoise, r.wsum, r.w2sum
        return res
