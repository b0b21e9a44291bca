"""C ABI checks that need no GPU: the library loads, exports every symbol
include/pk.h declares, sizes its buffers, and rejects bad arguments with
PK_EINVAL before any device work (validation-only context)."""

import ctypes
import os
import re

import pytest

from paper_1712_05834_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pk.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pk_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    decl = declared_symbols()
    assert len(decl) >= 13
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(_lib.EXPORTS)


def test_sizes():
    m = _lib.mesh_desc(64, 1000.0, "cic", False, True, "f8")
    assert _lib.mesh_bytes(m) == 64 ** 3 * 8
    m32 = _lib.mesh_desc(512, 1380.0, "tsc", True, True, "f4")
    assert _lib.mesh_bytes(m32) == 512 ** 3 * 4
    b = _lib.bin_desc(256, 0.0, 1.0, 5, (0, 2, 4), 2)
    assert _lib.result_doubles(b) == 256 * 4 + 256 * 5 + 2
    ws = _lib.workspace_bytes(m32, b, 10_000_000)
    assert ws >= 2 * 512 ** 3 * 4
    bad = _lib.mesh_desc(100, 1000.0)
    assert _lib.mesh_bytes(bad) == 0
    assert _lib.workspace_bytes(bad, b, 1) == 0


@pytest.fixture(scope="module")
def vctx():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.pk_ctx_create(ctypes.byref(h), -1, None) == _lib.PK_OK
    yield lib, h
    lib.pk_ctx_destroy(h)


def _paint(lib, h, m, pos=1, n=10, mesh=1, shift=0.0):
    return lib.pk_paint(h, ctypes.byref(m), ctypes.c_void_p(pos), None, n, shift,
                        ctypes.c_void_p(mesh), None)


def test_einval_before_device_work(vctx):
    lib, h = vctx
    good = _lib.mesh_desc(64, 1000.0, "cic")
    cases = [
        _lib.mesh_desc(63, 1000.0), _lib.mesh_desc(4, 1000.0), _lib.mesh_desc(4096, 1000.0),
        _lib.mesh_desc(64, 0.0), _lib.mesh_desc(64, -1.0), _lib.mesh_desc(64, float("nan")),
    ]
    for m in cases:
        assert _paint(lib, h, m) == _lib.PK_EINVAL
    m = _lib.mesh_desc(64, 1000.0)
    m.window = 5
    assert _paint(lib, h, m) == _lib.PK_EINVAL
    m = _lib.mesh_desc(64, 1000.0)
    m.reserved = 1
    assert _paint(lib, h, m) == _lib.PK_EINVAL
    assert _paint(lib, h, good, pos=0) == _lib.PK_EINVAL          # NULL pos with n > 0
    assert _paint(lib, h, good, n=-1) == _lib.PK_EINVAL
    assert _paint(lib, h, good, mesh=0) == _lib.PK_EINVAL
    assert _paint(lib, h, good, shift=float("inf")) == _lib.PK_EINVAL
    assert b"NULL" in lib.pk_last_error(h) or b"finite" in lib.pk_last_error(h)
    # valid arguments reach the device check of a validation-only context
    assert _paint(lib, h, good) == _lib.PK_EDEVICE


def test_bins_einval(vctx):
    lib, h = vctx
    inter = _lib.mesh_desc(64, 1000.0, "tsc", True)
    plain = _lib.mesh_desc(64, 1000.0, "tsc", False)
    res = ctypes.c_void_p(1)

    def bp(m, b):
        return lib.pk_bin_power(h, ctypes.byref(m), ctypes.byref(b), ctypes.c_void_p(1), res)

    assert bp(inter, _lib.bin_desc(33)) == _lib.PK_EINVAL          # above Nyquist, interlaced
    assert bp(plain, _lib.bin_desc(33)) == _lib.PK_EDEVICE         # allowed without interlacing
    assert bp(inter, _lib.bin_desc(32)) == _lib.PK_EDEVICE
    assert bp(inter, _lib.bin_desc(0)) == _lib.PK_EINVAL
    assert bp(inter, _lib.bin_desc(8, dk_f=0.0)) == _lib.PK_EINVAL
    assert bp(inter, _lib.bin_desc(8, kmin_f=-1.0)) == _lib.PK_EINVAL
    assert bp(inter, _lib.bin_desc(8, poles=(1,))) == _lib.PK_EINVAL  # odd ell
    assert bp(inter, _lib.bin_desc(8, poles=(2, 2))) == _lib.PK_EINVAL
    assert bp(inter, _lib.bin_desc(8, nmu=65)) == _lib.PK_EINVAL
    assert bp(inter, _lib.bin_desc(8, los=3)) == _lib.PK_EINVAL
    assert bp(plain, _lib.bin_desc(4000, dk_f=0.01, nmu=64)) == _lib.PK_EUNSUPPORTED


def test_fftpower_workspace_check(vctx):
    lib, h = vctx
    m = _lib.mesh_desc(32, 100.0, "cic")
    b = _lib.bin_desc(16)
    need = _lib.workspace_bytes(m, b, 100)
    st = lib.pk_fftpower(h, ctypes.byref(m), ctypes.byref(b), ctypes.c_void_p(1), None, 100,
                         ctypes.c_void_p(1), need - 1, ctypes.c_void_p(1))
    assert st == _lib.PK_EINVAL and b"workspace" in lib.pk_last_error(h)
    st = lib.pk_fftpower(h, ctypes.byref(m), ctypes.byref(b), ctypes.c_void_p(1), None, 100,
                         ctypes.c_void_p(1), need, ctypes.c_void_p(1))
    assert st == _lib.PK_EDEVICE


def test_null_context_and_create_errors():
    lib = _lib.load()
    m = _lib.mesh_desc(32, 100.0)
    assert lib.pk_fft_r2c(None, ctypes.byref(m), ctypes.c_void_p(1)) == _lib.PK_EINVAL
    assert lib.pk_ctx_create(None, 0, None) == _lib.PK_EINVAL
    assert lib.pk_last_error(None)


def test_bin_slots_must_fit_lds_beside_the_fused_xpass(vctx):
    """The exact bin sums take 16 bytes of LDS each (128-bit fixed point; the
    ell = 0 pole aliases the power sum and takes none).  Beside the float32
    x-pass at N = 1024 (90 KB of line buffers and tables) about 4600 sums fit
    the workgroup's 160 KB, beside the float64 one (108 KB) about 3300: 1000
    k-bins with ell = 0, 2, 4, 6 (4000 accumulated sums) fit the first only."""
    lib, h = vctx
    b = _lib.bin_desc(1000, 0.0, 1.0, 0, (0, 2, 4, 6), 2)
    res = ctypes.c_void_p(1)
    for dtype, want in (("f4", _lib.PK_EDEVICE), ("f8", _lib.PK_EUNSUPPORTED)):
        m = _lib.mesh_desc(1024, 1000.0, "cic", False, True, dtype)
        st = lib.pk_bin_power(h, ctypes.byref(m), ctypes.byref(b), ctypes.c_void_p(1), res)
        assert st == want, (dtype, st, lib.pk_last_error(h))


def test_lane_entry_points_validate(vctx):
    lib, h = vctx
    m = _lib.mesh_desc(32, 100.0, "cic")
    b = _lib.bin_desc(16)
    one = ctypes.c_void_p(1)
    # a validation-only context has no device, hence no lanes
    assert lib.pk_ctx_set_lanes(h, 2) == _lib.PK_EDEVICE
    assert lib.pk_ctx_set_lanes(h, 0) == _lib.PK_EINVAL
    assert lib.pk_ctx_set_lanes(h, _lib.PK_MAX_LANES + 1) == _lib.PK_EINVAL
    assert lib.pk_ctx_lanes(h) == 0
    assert lib.pk_fftpower_async(h, 0, ctypes.byref(m), ctypes.byref(b), one, None, 10, one,
                                 1 << 30, one) == _lib.PK_EINVAL
    assert lib.pk_lane_query(h, 0) == _lib.PK_EINVAL
    assert lib.pk_lane_wait(h, -1) == _lib.PK_EINVAL
    assert lib.pk_fftpower_batch(h, -1, None, None, None, None, None, None, 0, None) == _lib.PK_EINVAL
    assert lib.pk_fftpower_batch(h, 0, None, None, None, None, None, None, 0, None) == _lib.PK_EINVAL
    assert b"no lanes" in lib.pk_last_error(h)
    assert lib.pk_ctx_set_lanes(None, 1) == _lib.PK_EINVAL
    assert lib.pk_ctx_lanes(None) == 0


def test_survey_multipoles_validate(vctx):
    lib, h = vctx
    one = ctypes.c_void_p(1)
    obs = (ctypes.c_double * 3)(0.0, 0.0, -100.0)
    m = _lib.mesh_desc(32, 100.0, "tsc")
    b = _lib.bin_desc(16, poles=(0, 2, 4))
    need = _lib.convolved_workspace_bytes(m, b, 100, 300)
    assert need > 3 * _lib.mesh_bytes(m)
    assert _lib.convolved_doubles(b) == 3 * 16 + 4

    def call(m=m, b=b, obs=obs, nd=100, nr=300, wsb=need, dpos=one, rpos=one):
        return lib.pk_convolved_power(h, ctypes.byref(m), ctypes.byref(b), obs, dpos, None, nd,
                                      rpos, None, nr, one, wsb, one)

    assert call() == _lib.PK_EDEVICE  # valid: only the device is missing
    assert call(wsb=need - 1) == _lib.PK_EINVAL
    assert call(nd=0) == _lib.PK_EINVAL
    assert call(nr=0) == _lib.PK_EINVAL
    assert call(rpos=None) == _lib.PK_EINVAL
    assert call(obs=(ctypes.c_double * 3)(0.0, float("nan"), 0.0)) == _lib.PK_EINVAL
    assert call(b=_lib.bin_desc(16, poles=(0, 6))) == _lib.PK_EINVAL
    assert call(b=_lib.bin_desc(16, nmu=4, poles=(0,))) == _lib.PK_EINVAL
    assert call(b=_lib.bin_desc(16)) == _lib.PK_EINVAL  # no pole requested
    assert call(b=_lib.bin_desc(17, poles=(0,))) == _lib.PK_EINVAL  # top edge above N/2
    inter = _lib.mesh_desc(32, 100.0, "tsc", True)
    assert call(m=inter) == _lib.PK_EUNSUPPORTED
    assert _lib.convolved_workspace_bytes(m, _lib.bin_desc(17, poles=(0,)), 1, 1) == 0
    assert _lib.convolved_workspace_bytes(m, b, -1, 1) == 0
    res = _lib.Result()
    assert lib.pk_convolved_to_host(h, ctypes.byref(m), ctypes.byref(b), 0.0, one,
                                    ctypes.byref(res)) == _lib.PK_EINVAL


def test_sorted_paths_reject_more_than_int32_particles(vctx):
    # the sorted painting indexes records with 32-bit offsets: 2^31 particles
    # are refused before any device work (no workspace is even looked at)
    lib, h = vctx
    one = ctypes.c_void_p(1)
    m = _lib.mesh_desc(32, 100.0, "cic")
    b = _lib.bin_desc(16)
    big = 1 << 31
    st = lib.pk_fftpower(h, ctypes.byref(m), ctypes.byref(b), one, None, big, one, 1 << 62, one)
    assert st == _lib.PK_EUNSUPPORTED and b"2^31" in lib.pk_last_error(h)
    assert lib.pk_fftpower(h, ctypes.byref(m), ctypes.byref(b), one, None, big - 1, one,
                           1 << 62, one) == _lib.PK_EDEVICE
    bs = _lib.bin_desc(16, poles=(0,))
    obs = (ctypes.c_double * 3)(0.0, 0.0, -100.0)
    st = lib.pk_convolved_power(h, ctypes.byref(m), ctypes.byref(bs), obs, one, None, big // 2,
                                one, None, big // 2, one, 1 << 62, one)
    assert st == _lib.PK_EUNSUPPORTED


def test_c2r_validates(vctx):
    lib, h = vctx
    m = _lib.mesh_desc(32, 100.0)
    assert lib.pk_fft_c2r(h, ctypes.byref(m), None) == _lib.PK_EINVAL
    assert lib.pk_fft_c2r(h, ctypes.byref(m), ctypes.c_void_p(1)) == _lib.PK_EDEVICE
    bad = _lib.mesh_desc(24, 100.0)
    assert lib.pk_fft_c2r(h, ctypes.byref(bad), ctypes.c_void_p(1)) == _lib.PK_EINVAL


def test_shape_spectrum_validates(vctx):
    lib, h = vctx
    m = _lib.mesh_desc(32, 100.0)
    need = _lib.shape_table_len(m)
    assert need == 3 * 16 ** 2 + 1
    one = ctypes.c_void_p(1)
    assert lib.pk_shape_spectrum(h, ctypes.byref(m), one, one, need - 1) == _lib.PK_EINVAL
    assert lib.pk_shape_spectrum(h, ctypes.byref(m), None, one, need) == _lib.PK_EINVAL
    assert lib.pk_shape_spectrum(h, ctypes.byref(m), one, one, need) == _lib.PK_EDEVICE
    assert _lib.shape_table_len(_lib.mesh_desc(24, 1.0)) == 0


def test_num_kbins_sizing_query():
    # whole bins [kmin + b dk, kmin + (b + 1) dk) with the top edge <= kmax
    # (FFTPower k-bins, Sec. 3.4.1), in units of k_f
    lib = _lib.load()
    assert lib.pk_num_kbins(0.0, 1.0, 32.0) == 32        # up to the Nyquist index of 64^3
    assert lib.pk_num_kbins(0.0, 1.0, 32.5) == 32
    assert lib.pk_num_kbins(0.5, 1.5, 8.0) == 5          # 0.5 + 5 * 1.5 = 8 exactly
    assert lib.pk_num_kbins(0.5, 1.5, 7.99) == 4
    assert lib.pk_num_kbins(0.0, 0.1, 0.3) == 3          # 3 * 0.1 is 0.30000000000000004
    assert lib.pk_num_kbins(0.0, 2.0, 1.0) == 0          # no whole bin fits
    for bad in ((-1.0, 1.0, 4.0), (0.0, 0.0, 4.0), (0.0, -1.0, 4.0), (4.0, 1.0, 4.0),
                (0.0, float("nan"), 4.0), (0.0, 1.0, float("inf"))):
        assert lib.pk_num_kbins(*bad) == _lib.PK_EINVAL, bad
    assert lib.pk_num_kbins(0.0, 1.0, 5000.0) == _lib.PK_EUNSUPPORTED
    assert _lib.num_kbins(0.0, 1.0, 256.0) == 256
    with pytest.raises(ValueError):
        _lib.num_kbins(0.0, 0.0, 1.0)


def test_binding_refuses_host_and_mistyped_tensors_before_any_launch():
    # The library dereferences raw device addresses: a host tensor, a tensor
    # of the wrong dtype or a short buffer must be refused by the binding
    # (ValueError) before the C call, not become a device memory fault.
    import torch

    ctx = _lib.Context(_lib.PK_DEVICE_NONE)
    m = _lib.mesh_desc(32, 100.0, "cic", False, True, "f4")
    b = _lib.bin_desc(16, 0.0, 1.0, 0, (0,), 2)
    pos = torch.zeros((10, 3), dtype=torch.float32)
    with pytest.raises(ValueError, match="GPU"):
        ctx.pk_fftpower(m, b, pos, None, 10, torch.zeros(8, dtype=torch.uint8),
                        torch.zeros(_lib.result_doubles(b), dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU"):
        ctx.pk_paint(m, pos, torch.ones(10), 10, 0.0, torch.zeros(32 ** 3))
    with pytest.raises(ValueError, match="GPU"):
        ctx.pk_bin_power(m, b, torch.zeros(32 ** 3), torch.zeros(_lib.result_doubles(b),
                                                                  dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU"):
        ctx.pk_result_to_host(m, b, torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="required"):
        ctx.pk_fftpower(m, b, None, None, 10, None, None)
    with pytest.raises(ValueError):
        ctx.pk_fftpower_batch([m], [b], [pos], [None], [10], [], [None])
    with pytest.raises(TypeError):
        ctx.pk_fft_r2c(m, [0.0] * 8)
    # the front end refuses a host weight next to device positions before
    # building anything (checked without a device: a host pos is refused too)
    from paper_1712_05834_amd import api

    with pytest.raises(ValueError):
        api.CatalogMesh(pos, 32, 100.0, weight=torch.ones(10))
    ctx.close()



def test_tuning_table_entry_points_validate():
    ctx = _lib.Context(_lib.PK_DEVICE_NONE)
    with pytest.raises(_lib.PkError):
        ctx.pk_ctx_set_autotune(2)
    ctx.pk_ctx_set_autotune(1)
    good = {"nmesh": 128, "dtype": 0, "window": 3, "interlaced": 1, "density": -3,
            "split": 1, "xpass_per_cu": 1, "ms": 0.5}
    ctx.tune_load([good])
    assert ctx.tune_table() == [good]
    for key, bad in (("split", 2), ("split", -1), ("xpass_per_cu", 3), ("nmesh", 100),
                     ("window", 5)):
        with pytest.raises(_lib.PkError):
            ctx.tune_load([{**good, key: bad}])
    # an entry with the same key replaces the old one
    ctx.tune_load([{**good, "split": 0}])
    assert len(ctx.tune_table()) == 1 and ctx.tune_table()[0]["split"] == 0
    ctx.close()
