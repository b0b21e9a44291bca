"""Bitwise reproducibility of the bin sums (FFTPower binning, Sec. 3.4.1)
and of the fused painting (Sec. 3.3.1, Eq. 1).

Every bin sum is an exact 128-bit fixed-point sum (the per-mode terms are
truncated once to a grid set by an a-priori bound; integer addition does not
depend on order), and the per-workgroup partial rows are added exactly too.
So the binning of a given spectrum gives the same bits on every call,
whatever the order in which lanes and workgroups add and however many
workgroups there are.  The fused painting of pk_fftpower adds its terms as
64-bit fixed-point integers on one scale for the whole mesh, so each cell is
the same whatever the order of its adds and whatever the tiling; with the
deterministic FFT passes pk_fftpower gives the same bits on every call."""

import numpy as np
import pytest
import torch

from paper_1712_05834_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _spectrum(ctx, n, dtype, seed):
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    mesh = torch.randn((n, n, n), generator=g, device="cuda:0", dtype=torch.float64)
    mesh = mesh.to(torch.float32 if dtype == "f4" else torch.float64)
    m = _lib.mesh_desc(n, 500.0, "pcs", True, True, dtype)
    ctx.pk_fft_r2c(m, mesh)
    return m, mesh


@pytest.mark.parametrize("dtype", ["f4", "f8"])
@pytest.mark.parametrize("n", [32, 128])
def test_bin_power_twice_is_bitwise_equal(ctx, dtype, n):
    m, spec = _spectrum(ctx, n, dtype, seed=n)
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 5, (0, 2, 4, 6), 2)
    r1 = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    r2 = torch.empty_like(r1)
    ctx.pk_bin_power(m, b, spec, r1)
    ctx.pk_bin_power(m, b, spec, r2)
    torch.cuda.synchronize()
    assert torch.equal(r1[:-2], r2[:-2])
    assert bool(torch.isfinite(r1[:-2]).all())


def test_cross_power_binning_is_bitwise_equal(ctx):
    m, s1 = _spectrum(ctx, 64, "f4", seed=1)
    _, s2 = _spectrum(ctx, 64, "f4", seed=2)
    b = _lib.bin_desc(32, 0.0, 1.0, 3, (0, 2), 1)
    r1 = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    r2 = torch.empty_like(r1)
    ctx.pk_bin_cross(m, b, s1, s2, r1)
    ctx.pk_bin_cross(m, b, s1, s2, r2)
    torch.cuda.synchronize()
    assert torch.equal(r1[:-2], r2[:-2])


def test_binning_of_a_non_finite_spectrum_is_nan(ctx):
    # a NaN mode must not turn into a finite sum through the fixed point
    m, spec = _spectrum(ctx, 32, "f4", seed=3)
    spec.view(-1)[1058] = float("nan")  # Re c(kx = 1, ky = 1, kz = 1), inside the binning
    b = _lib.bin_desc(16, 0.0, 1.0, 0, (0, 2), 2)
    r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_bin_power(m, b, spec, r)
    torch.cuda.synchronize()
    assert bool(torch.isnan(r[:-2]).any())


@pytest.mark.parametrize("window", ["cic", "tsc", "pcs"])
@pytest.mark.parametrize("weighted", [False, True])
def test_fused_path_twice_is_bitwise_equal(ctx, window, weighted):
    # pk_fftpower twice on one catalog (clustered, so that many adds meet in
    # one cell): the same bits, the painted mesh included
    n, box, npart = 128, 700.0, 300_000
    rng = np.random.default_rng(7)
    centres = rng.uniform(0, box, (300, 3))
    pos = (centres[rng.integers(0, 300, npart)] + rng.normal(0, 3.0, (npart, 3))) % box
    pos = torch.from_numpy(pos.astype(np.float32)).to("cuda:0")
    w = (torch.from_numpy(rng.uniform(0.1, 3.0, npart).astype(np.float32)).to("cuda:0")
         if weighted else None)
    m = _lib.mesh_desc(n, box, window, True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 4, (0, 2, 4), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")
    rs, meshes = [], []
    for _ in range(2):
        r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
        ctx.pk_fftpower(m, b, pos, w, npart, ws, r)
        torch.cuda.synchronize()
        rs.append(r.clone())
        meshes.append(ws.clone())
    assert torch.equal(rs[0], rs[1])
    assert bool(torch.isfinite(rs[0][:-2]).all())
    del meshes


def test_fused_path_with_a_non_finite_weight_is_nan(ctx):
    # the fixed-point painting must not turn a NaN amount into finite cells
    n, box, npart = 32, 100.0, 5000
    rng = np.random.default_rng(8)
    pos = torch.from_numpy(rng.uniform(0, box, (npart, 3)).astype(np.float32)).to("cuda:0")
    w = torch.ones(npart, dtype=torch.float32, device="cuda:0")
    w[17] = float("nan")
    m = _lib.mesh_desc(n, box, "cic", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")
    r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower(m, b, pos, w, npart, ws, r)
    torch.cuda.synchronize()
    assert bool(torch.isnan(r[: b.nk]).all())


@pytest.mark.parametrize("scale", [2.0 ** 45, 2.0 ** -40, 1e12, 1e-12])
def test_fused_path_does_not_depend_on_the_weight_scale(ctx, scale):
    # P = |F|^2 / (sum w)^2 and the shot noise are invariant under w -> s w.
    # The exact painting sets its grid 2^-S from n and sum w^2 (S = 42 at unit
    # weights here), so these scales take it to S = -3 and S = 82; with s a
    # power of two the painted integers are the same and so is every bit of
    # the normalised result.  (The float32 spectrum bounds the range: the
    # compensated |F|^2 of every mode must stay a normal float32.)
    n, box, npart = 64, 400.0, 50_000
    rng = np.random.default_rng(11)
    pos = torch.from_numpy(rng.uniform(0, box, (npart, 3)).astype(np.float32)).to("cuda:0")
    w0 = rng.uniform(0.5, 1.5, npart).astype(np.float32)
    m = _lib.mesh_desc(n, box, "tsc", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 3, (0, 2), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")

    def run(w):
        wt = torch.from_numpy(w).to("cuda:0")
        r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
        ctx.pk_fftpower(m, b, pos, wt, npart, ws, r)
        out = ctx.pk_result_to_host(m, b, r)
        torch.cuda.synchronize()
        return out

    ref = run(w0)
    got = run((w0.astype(np.float64) * scale).astype(np.float32))
    exact = scale in (2.0 ** 45, 2.0 ** -40)
    rtol = 1e-12 if exact else 1e-5
    ok, ok2 = ref["modes"] > 0, ref["modes2d"] > 0
    np.testing.assert_array_equal(got["modes"], ref["modes"])
    assert np.isfinite(got["power"][ok]).all() and np.isfinite(got["power2d"][ok2]).all()
    np.testing.assert_allclose(got["power"][ok], ref["power"][ok], rtol=rtol)
    np.testing.assert_allclose(got["poles"][2][ok], ref["poles"][2][ok],
                               rtol=0, atol=rtol * np.abs(ref["power"][ok]).max())
    np.testing.assert_allclose(got["power2d"][ok2], ref["power2d"][ok2], rtol=10 * rtol)
    np.testing.assert_allclose(got["shotnoise"], ref["shotnoise"], rtol=rtol)
