"""GPU parity of every libpk entry point against the CPU float64 oracle.

Tolerances (float32 path): per bin |dP| / |P| <= 1e-5 for P(k) and P(k, mu);
|dP_ell| <= 1e-5 |P_0| for ell > 0 (P_ell can cross zero); float64 path: the
same definitions at 1e-12.  Mode counts are compared bit for bit.  Meshes are
compared cell by cell against the oracle's painted mesh, spectra mode by mode
against the oracle's r2c.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, api, synth
from tests import packing
from tests.powercheck import check_power

pytestmark = pytest.mark.gpu

TOL = {"f8": 1e-12, "f4": 1e-5}
TDT = {"f8": torch.float64, "f4": torch.float32}
NDT = {"f8": np.float64, "f4": np.float32}


@pytest.fixture(scope="module")
def ctx():
    props = torch.cuda.get_device_properties(0)
    print(f"\ndevice: {props.name}, {props.total_memory / 2**30:.0f} GiB, "
          f"{props.multi_processor_count} CUs", flush=True)
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# ------------------------------------------------------------------ painting

@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("shift,weighted", [(0.0, False), (0.5, True)])
def test_paint_matches_oracle(ctx, dtype, order, shift, weighted):
    n, box, npart = 32, 250.0, 12345
    rng = np.random.default_rng(order * 10 + int(weighted))
    pos = rng.uniform(-0.5 * box, 1.5 * box, (npart, 3)).astype(NDT[dtype])
    w = synth.uniform_weights(npart, seed=5).astype(NDT[dtype]) if weighted else None
    m = _lib.mesh_desc(n, box, order, False, True, dtype)
    mesh = torch.empty((n, n, n), dtype=TDT[dtype], device="cuda:0")
    wsums = torch.empty(2, dtype=torch.float64, device="cuda:0")
    ctx.pk_paint(m, dev(pos), None if w is None else dev(w), npart, shift, mesh, wsums)
    got = mesh.cpu().numpy().astype(np.float64)
    want = oracle.paint_mesh(pos.astype(np.float64), n, box, order,
                             None if w is None else w.astype(np.float64), shift)
    tol = 1e-13 if dtype == "f8" else 2e-6
    assert np.abs(got - want).max() <= tol * np.abs(want).max()
    ws = np.ones(npart) if w is None else w.astype(np.float64)
    np.testing.assert_allclose(wsums.cpu().numpy(), [ws.sum(), (ws * ws).sum()], rtol=1e-12)


def test_paint_empty_catalog(ctx):
    m = _lib.mesh_desc(16, 10.0, "tsc", False, True, "f4")
    mesh = torch.full((16, 16, 16), 7.0, dtype=torch.float32, device="cuda:0")
    wsums = torch.full((2,), 3.0, dtype=torch.float64, device="cuda:0")
    ctx.pk_paint(m, None, None, 0, 0.0, mesh, wsums)
    assert float(mesh.abs().max()) == 0.0 and float(wsums.abs().max()) == 0.0


# ------------------------------------------------------------------ r2c FFT

# Error bars of the transform.
# * Per mode, on a zero-mean field (all modes of comparable size): a radix-2^r
#   Stockham FFT with accurate twiddles has a relative rms error of about
#   eps sqrt(log2 L) per line of L points (each of the log2 L butterfly
#   levels adds a rounding of relative size ~eps, incoherently); the 3-D
#   transform has log2 N^3 levels.  The bar allows 3x that rms, and for the
#   largest single-mode error 8x (the maximum of N^3 / 2 roughly Gaussian
#   errors is ~6 rms at 512^3).  Errors are per mode against the rms
#   amplitude.
# * Normwise, on a field with a large mean (0.3 per cell): the error of a
#   floating-point FFT is bounded in norm, ||dc||_2 <= log2(N^3) eta ||c||_2
#   with eta a small multiple of eps (Higham, Accuracy and Stability of
#   Numerical Algorithms, 2nd ed., Sec. 24.1).  ||c|| is then dominated by
#   the DC mode, and single modes may carry errors of order eps |DC|: the
#   real-input split forms c(.,.,N/2) of each column as the difference of two
#   sums of about N/2 values each, which cancel to the size of the
#   fluctuations.  The bar is ||dc|| / ||c|| <= 2 eps log2(N^3).
EPS = {"f8": 2.0 ** -53, "f4": 2.0 ** -24}


def _r2c_pair(ctx, f, dtype):
    n = f.shape[0]
    m = _lib.mesh_desc(n, 1.0, "cic", False, True, dtype)
    mesh = dev(f)
    ctx.pk_fft_r2c(m, mesh)
    got = packing.unpack(packing.as_complex(mesh.cpu().numpy().astype(np.float64)))
    del mesh
    return got, oracle.r2c(f.astype(np.float64))


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512])
def test_fft_r2c_matches_oracle_per_mode(ctx, dtype, n):
    f = np.random.default_rng(n).standard_normal((n, n, n)).astype(NDT[dtype])
    got, want = _r2c_pair(ctx, f, dtype)
    rms = math.sqrt(np.mean(np.abs(want) ** 2))
    d = np.abs(got - want) / rms
    err_rms, err_max = math.sqrt(np.mean(d ** 2)), d.max()
    bound = EPS[dtype] * math.sqrt(math.log2(n ** 3))
    print(f"n={n} {dtype}: per-mode error / rms amplitude: rms {err_rms:.2e}, max {err_max:.2e}; "
          f"eps sqrt(log2 N^3) = {bound:.2e}")
    assert err_rms <= 3 * bound and err_max <= 8 * bound, (err_rms, err_max, bound)


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("n", [16, 64, 256])
def test_fft_r2c_normwise_with_large_mean(ctx, dtype, n):
    f = (np.random.default_rng(n + 1).standard_normal((n, n, n)) + 0.3).astype(NDT[dtype])
    got, want = _r2c_pair(ctx, f, dtype)
    norm_err = math.sqrt(np.sum(np.abs(got - want) ** 2) / np.sum(np.abs(want) ** 2))
    bound = 2 * EPS[dtype] * math.log2(n ** 3)
    print(f"n={n} {dtype}: normwise error {norm_err:.2e}, bound 2 eps log2 N^3 = {bound:.2e}")
    assert norm_err <= bound, (norm_err, bound)


def test_fft_r2c_plane_wave(ctx):
    n = 64
    x = np.arange(n)
    g = np.meshgrid(x, x, x, indexing="ij")
    f = np.cos(2 * np.pi * (5 * g[0] - 3 * g[1] + 7 * g[2]) / n)
    m = _lib.mesh_desc(n, 1.0, "cic", False, True, "f8")
    mesh = dev(f)
    ctx.pk_fft_r2c(m, mesh)
    c = packing.unpack(packing.as_complex(mesh.cpu().numpy()))
    assert abs(c[5, (-3) % n, 7] - n ** 3 / 2) < 1e-8
    c[5, (-3) % n, 7] = 0
    assert np.abs(c).max() < 1e-8


def test_fft_is_deterministic(ctx):
    n = 128
    f = np.random.default_rng(3).standard_normal((n, n, n)).astype(np.float32)
    m = _lib.mesh_desc(n, 1.0, "cic", False, True, "f4")
    a, b = dev(f), dev(f)
    ctx.pk_fft_r2c(m, a)
    ctx.pk_fft_r2c(m, b)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ compensate

@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_compensate_matches_oracle(ctx, dtype, order):
    n = 32
    rng = np.random.default_rng(order)
    ca = oracle.r2c(rng.standard_normal((n, n, n)))
    cb = oracle.r2c(rng.standard_normal((n, n, n)))
    m = _lib.mesh_desc(n, 1.0, order, True, True, dtype)
    ta = dev(packing.to_real_view(packing.pack(ca), NDT[dtype]))
    tb = dev(packing.to_real_view(packing.pack(cb), NDT[dtype]))
    ctx.pk_compensate(m, ta, tb)
    got = packing.unpack(packing.as_complex(ta.cpu().numpy().astype(np.float64)))
    want = oracle.compensate(oracle.interlace_combine(ca, cb, n), n, order)
    # the packed column cannot hold the non-Hermitian interlaced values of the
    # kz = N/2 plane or of plane-0 modes on a Nyquist index; none of them is
    # ever binned for interlaced meshes (top edge <= N/2)
    nx, ny, nz = oracle.mode_indices(n)
    skip = (((np.abs(nx)[:, None, None] == n // 2) | (np.abs(ny)[None, :, None] == n // 2))
            & (nz == 0)[None, None, :]) | (nz == n // 2)[None, None, :]
    tol = 1e-12 if dtype == "f8" else 2e-6
    err = np.abs(got - want)[~skip].max() / np.abs(want).max()
    assert err <= tol, err


# ------------------------------------------------------------------ binning

@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("nmu,poles,los", [(0, (), 2), (5, (0, 2, 4), 2), (3, (2, 0, 6), 0)])
def test_bin_power_matches_oracle(ctx, dtype, nmu, poles, los):
    n, box = 64, 700.0
    f = synth.fixed_amplitude_field(n, box, synth.pk_lognormal_c2, seed=4)
    f += 0.05 * np.random.default_rng(1).standard_normal(f.shape)  # break isotropy a little
    c = oracle.r2c(f)
    wsum, w2sum = float(n ** 3), 123.0
    want = oracle.fftpower_from_spectra(c, None, n, box, 2, False, wsum, w2sum, 1, nmu=nmu,
                                        poles=poles, los=los)
    m = _lib.mesh_desc(n, box, "cic", False, False, dtype)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, nmu, poles, los)
    spec = dev(packing.to_real_view(packing.pack(c), NDT[dtype]))
    res = torch.zeros(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power(m, b, spec, res)
    res[-2] = wsum
    res[-1] = w2sum
    got = ctx.pk_result_to_host(m, b, res)
    check_power(got, want, TOL[dtype], f"{dtype} nmu={nmu} poles={poles} los={los}")


def test_bin_power_general_edges(ctx):
    n, box = 32, 300.0
    f = np.random.default_rng(8).standard_normal((n, n, n)) + 1.0
    c = oracle.r2c(f)
    kw = dict(kmin_f=0.5, dk_f=1.5, nk=9, nmu=4, poles=(0, 2), los=1)
    want = oracle.fftpower_from_spectra(c, None, n, box, 2, False, 10.0, 2.0, 1, **kw)
    m = _lib.mesh_desc(n, box, "cic", False, False, "f8")
    b = _lib.bin_desc(9, 0.5, 1.5, 4, (0, 2), 1)
    spec = dev(packing.to_real_view(packing.pack(c), np.float64))
    res = torch.zeros(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power(m, b, spec, res)
    res[-2], res[-1] = 10.0, 2.0
    check_power(ctx.pk_result_to_host(m, b, res), want, 1e-12, "general edges")


# ------------------------------------------------------------------ end to end

def _run_fftpower(ctx, pos, weight, n, box, window, inter, comp, dtype, b):
    m = _lib.mesh_desc(n, box, window, inter, comp, dtype)
    ws = torch.empty(_lib.workspace_bytes(m, b, len(pos)), dtype=torch.uint8, device="cuda:0")
    res = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower(m, b, dev(pos), None if weight is None else dev(weight), len(pos), ws, res)
    return ctx.pk_result_to_host(m, b, res)


def test_fftpower_plain_fp64_64cube(ctx):
    """10^4 uniform particles, L = 1000, CIC on 64^3, float64, 1-D P(k)."""
    pos = synth.uniform_catalog(10_000, 1000.0, seed=1)
    b = _lib.bin_desc(32)
    got = _run_fftpower(ctx, pos, None, 64, 1000.0, "cic", False, True, "f8", b)
    want = oracle.fftpower(pos, 64, 1000.0, "cic")
    check_power(got, want, 1e-12, "plain fp64")
    golden = np.loadtxt("tests/golden/modecounts_n64_dk1.txt", dtype=np.int64)
    np.testing.assert_array_equal(got["modes"], golden)


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("window,inter", [("cic", True), ("tsc", True), ("pcs", False),
                                          ("pcs", True), ("tsc", False)])
@pytest.mark.parametrize("n", [16, 64])
def test_fftpower_matrix(ctx, dtype, window, inter, n):
    box = 400.0
    npart = 20_011
    pos = synth.uniform_catalog(npart, box, seed=n + 3).astype(NDT[dtype])
    w = synth.uniform_weights(npart, seed=9).astype(NDT[dtype])
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 5, (0, 2, 4), 2)
    got = _run_fftpower(ctx, pos, w, n, box, window, inter, True, dtype, b)
    want = oracle.fftpower(pos.astype(np.float64), n, box, window, inter, True,
                           w.astype(np.float64), nmu=5, poles=(0, 2, 4))
    check_power(got, want, TOL[dtype], f"{dtype} {window} inter={inter} n={n}")


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("window", ["cic", "tsc"])
def test_fftpower_wraps_positions_and_piles_up(ctx, dtype, window):
    # the fused path (bucketing, sorted painting) with positions in [-L, 2L),
    # values on the box edges (0, +-L, 2L and just below L) and 300 particles
    # in one spot: periodic wrap and a dense cell against the oracle
    n, box = 32, 100.0
    rng = np.random.default_rng(61)
    pos = rng.uniform(-box, 2 * box, (4000, 3))
    edges = np.array([0.0, box, -box, 2 * box, box * (1 - 2.0 ** -50), 0.5 * box])
    special = np.stack(np.meshgrid(edges, edges, edges, indexing="ij"), axis=-1).reshape(-1, 3)
    pile = np.tile([[37.3, 12.9, 81.05]], (300, 1))
    pos = np.concatenate([pos, special, pile]).astype(NDT[dtype])
    w = rng.uniform(0.5, 1.5, len(pos)).astype(NDT[dtype])
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 3, (0, 2), 2)
    got = _run_fftpower(ctx, pos, w, n, box, window, True, True, dtype, b)
    want = oracle.fftpower(pos.astype(np.float64), n, box, window, True, True,
                           w.astype(np.float64), nmu=3, poles=(0, 2))
    check_power(got, want, TOL[dtype], f"{dtype} {window} wrap + pile-up")


def test_fftpower_uncompensated_los_x(ctx):
    box, n = 200.0, 32
    pos = synth.uniform_catalog(5000, box, seed=77)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 2, (2,), 0)
    got = _run_fftpower(ctx, pos, None, n, box, "tsc", True, False, "f8", b)
    want = oracle.fftpower(pos, n, box, "tsc", True, False, nmu=2, poles=(2,), los=0)
    check_power(got, want, 1e-12, "uncompensated los=x")


def test_fftpower_reuses_tables_and_repeats(ctx):
    n, box = 64, 800.0
    pos = synth.uniform_catalog(30_000, box, seed=5).astype(np.float32)
    b = _lib.bin_desc(32, 0.0, 1.0, 0, (0, 2), 2)
    r1 = _run_fftpower(ctx, pos, None, n, box, "cic", True, True, "f4", b)
    before = ctx.table_bytes()
    r2 = _run_fftpower(ctx, pos, None, n, box, "cic", True, True, "f4", b)
    assert ctx.table_bytes() == before
    np.testing.assert_array_equal(r1["modes"], r2["modes"])
    np.testing.assert_allclose(r1["power"], r2["power"], rtol=1e-6, equal_nan=True)


def test_api_front_end(ctx):
    box, n = 500.0, 32
    pos = synth.uniform_catalog(4000, box, seed=12)
    mesh = api.to_mesh(dev(pos), n, box, resampler="tsc", interlaced=True, dtype="f8")
    r = api.FFTPower(mesh, mode="2d", Nmu=4, poles=[0, 2])
    want = oracle.fftpower(pos, n, box, "tsc", True, nmu=4, poles=(0, 2))
    check_power(r, want, 1e-12, "api")
    painted, wsums = mesh.paint()
    np.testing.assert_allclose(painted.cpu().numpy(), oracle.paint_mesh(pos, n, box, 3),
                               atol=1e-12)


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("window,inter", [("cic", True), ("tsc", False)])
def test_fftpower_catalog_order_routes_agree(ctx, dtype, window, inter):
    # The bucketing takes one of two routes, chosen on the device from the
    # order of the catalog: in column order (runs of equal columns) or not
    # (slab partition).  The same weighted catalog, sorted by column and
    # shuffled, must give the same spectra, both matching the oracle.
    n, box, npart = 64, 500.0, 120_000
    rng = np.random.default_rng(2024)
    pos = rng.uniform(0.0, box, (npart, 3)).astype(NDT[dtype]).astype(np.float64)
    w = rng.uniform(0.5, 1.5, npart).astype(NDT[dtype]).astype(np.float64)
    cell = np.floor(pos / (box / n)).astype(np.int64) % n
    by_column = np.lexsort((cell[:, 2], cell[:, 1], cell[:, 0]))
    shuffled = rng.permutation(npart)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 3, (0, 2), 2)
    res = {}
    for name, idx in (("column order", by_column), ("shuffled", shuffled)):
        res[name] = _run_fftpower(ctx, pos[idx].astype(NDT[dtype]), w[idx].astype(NDT[dtype]),
                                  n, box, window, inter, True, dtype, b)
    want = oracle.fftpower(pos, n, box, window, inter, True, w, nmu=3, poles=(0, 2))
    for name, got in res.items():
        check_power(got, want, TOL[dtype], f"{dtype} {window} {name}")
    a, s = res["column order"], res["shuffled"]
    np.testing.assert_array_equal(a["modes"], s["modes"])
    ok = a["modes"] > 0
    rtol = 1e-13 if dtype == "f8" else 1e-6
    np.testing.assert_allclose(s["power"][ok], a["power"][ok], rtol=rtol)
    assert s["shotnoise"] == pytest.approx(a["shotnoise"], rel=1e-12)


@pytest.mark.parametrize("dtype", ["f8", "f4"])
def test_fftpower_shuffled_catalog_in_one_slab(ctx, dtype):
    # A catalog in random order whose particles all lie in one x-slab (and
    # a few in a second one): the bucketing's slab route then has one slab
    # holding nearly everything and N - 2 empty slabs.
    n, box, npart = 32, 320.0, 60_000
    h = box / n
    rng = np.random.default_rng(77)
    pos = rng.uniform(0.0, box, (npart, 3))
    pos[:, 0] = rng.uniform(5 * h, 6 * h, npart)
    pos[:100, 0] = rng.uniform(20 * h, 21 * h, 100)
    pos = pos[rng.permutation(npart)].astype(NDT[dtype])
    w = rng.uniform(0.5, 1.5, npart).astype(NDT[dtype])
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 2, (0, 2), 2)
    got = _run_fftpower(ctx, pos, w, n, box, "tsc", True, True, dtype, b)
    want = oracle.fftpower(pos.astype(np.float64), n, box, "tsc", True, True,
                           w.astype(np.float64), nmu=2, poles=(0, 2))
    check_power(got, want, TOL[dtype], f"{dtype} one slab")
