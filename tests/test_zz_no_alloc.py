"""pk_bin_power_noalloc (the binning entry point that allocates nothing and
keeps its partial sums in fixed device memory) against pk_bin_power on the
same spectra, called twice in a row, the second time with a smaller mesh and
binning, so that whatever the first call left in the fixed memory must not
leak into the second.  Bar: the sums are equal bit for bit (both are exact
128-bit fixed-point sums on the same scale, so the smaller grid of the fixed
memory does not change them); the two weight slots are left untouched by
both."""

import numpy as np
import pytest
import torch

from paper_1712_05834_amd import _lib

pytestmark = pytest.mark.gpu

TDT = {"f8": torch.float64, "f4": torch.float32}


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _spectrum(ctx, n, dtype, seed):
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    mesh = torch.randn((n, n, n), generator=g, device="cuda:0", dtype=torch.float64).to(TDT[dtype])
    m = _lib.mesh_desc(n, 700.0, "tsc", False, False, dtype)
    ctx.pk_fft_r2c(m, mesh)
    return m, mesh


def _both(ctx, m, b, spec):
    sentinel = torch.tensor([12.5, -3.25], dtype=torch.float64, device="cuda:0")
    want = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    got = torch.full_like(want, float("nan"))
    want[-2:] = sentinel
    got[-2:] = sentinel
    ctx.pk_bin_power(m, b, spec, want)
    ctx.pk_bin_power_noalloc(m, b, spec, got)
    torch.cuda.synchronize()
    w, g_ = want.cpu().numpy(), got.cpu().numpy()
    assert np.array_equal(g_[-2:], sentinel.cpu().numpy()), "weight slots changed"
    assert np.array_equal(w[:-2].view(np.uint64), g_[:-2].view(np.uint64)), "sums differ"
    return 0.0


@pytest.mark.parametrize("dtype", ["f4", "f8"])
def test_noalloc_binning_matches_pk_bin_power_twice(ctx, dtype):
    # first call: 64^3, P(k, mu) with 4 mu bins and ell = 0, 2, 4, 6
    m1, s1 = _spectrum(ctx, 64, dtype, seed=1)
    b1 = _lib.bin_desc(32, 0.0, 1.0, 4, (0, 2, 4, 6), 2)
    e1 = _both(ctx, m1, b1, s1)
    # second call, smaller: 32^3, non-integer edges (the device edge table),
    # line of sight x, fewer slots
    m2, s2 = _spectrum(ctx, 32, dtype, seed=2)
    b2 = _lib.bin_desc(9, 0.5, 1.5, 0, (2,), 0)
    e2 = _both(ctx, m2, b2, s2)
    assert e1 == 0.0 and e2 == 0.0
    # and the finalised spectra agree
    res = torch.empty(_lib.result_doubles(b2), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power_noalloc(m2, b2, s2, res)
    res[-2:] = torch.tensor([float(32 ** 3), float(32 ** 3)], dtype=torch.float64)
    got = ctx.pk_result_to_host(m2, b2, res)
    ctx.pk_bin_power(m2, b2, s2, res)
    want = ctx.pk_result_to_host(m2, b2, res)
    np.testing.assert_array_equal(got["modes"], want["modes"])
    ok = want["modes"] > 0
    assert np.array_equal(got["power"][ok], want["power"][ok])
    assert np.array_equal(got["poles"][2][ok], want["poles"][2][ok])


def test_noalloc_refuses_bad_arguments_before_launch(ctx):
    m = _lib.mesh_desc(32, 100.0, "cic", False, False, "f4")
    b = _lib.bin_desc(16, 0.0, 1.0, 0, (0,), 2)
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    lib = _lib.load()
    import ctypes

    st = lib.pk_bin_power_noalloc(ctx.handle, ctypes.byref(m), ctypes.byref(b), None,
                                  ctypes.c_void_p(res.data_ptr()))
    assert st == _lib.PK_EINVAL
    bad = _lib.bin_desc(16, 0.0, 1.0, 0, (1,), 2)  # odd multipole
    mesh = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda:0")
    st = lib.pk_bin_power_noalloc(ctx.handle, ctypes.byref(m), ctypes.byref(bad),
                                  ctypes.c_void_p(mesh.data_ptr()),
                                  ctypes.c_void_p(res.data_ptr()))
    assert st == _lib.PK_EINVAL
