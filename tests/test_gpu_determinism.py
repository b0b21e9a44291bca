"""Bitwise reproducibility of the bin sums (FFTPower binning, Sec. 3.4.1).

Every bin sum is an exact 128-bit fixed-point sum (the per-mode terms are
truncated once to a grid set by an a-priori bound; integer addition does not
depend on order), and the per-workgroup partial rows are added exactly too.
So the binning of a given spectrum gives the same bits on every call,
whatever the order in which lanes and workgroups add and however many
workgroups there are.  The painting adds float64 terms in LDS in no fixed
order and is not covered: pk_fftpower is reproducible to rounding only."""

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


def test_fused_path_repeats_to_rounding_of_the_painting(ctx):
    # pk_fftpower twice on one catalog: the binning is exact, the painting's
    # float64 LDS sums are not in a fixed order; the results agree to the
    # float32 bar (they usually agree bit for bit)
    n, box = 128, 700.0
    rng = np.random.default_rng(7)
    pos = torch.from_numpy(rng.uniform(0, box, (200_000, 3)).astype(np.float32)).to("cuda:0")
    m = _lib.mesh_desc(n, box, "tsc", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 4, (0, 2, 4), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, 200_000), dtype=torch.uint8, device="cuda:0")
    outs = []
    for _ in range(2):
        r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
        ctx.pk_fftpower(m, b, pos, None, 200_000, ws, r)
        outs.append(ctx.pk_result_to_host(m, b, r))
    ok = outs[0]["modes"] > 0
    np.testing.assert_allclose(outs[0]["power"][ok], outs[1]["power"][ok], rtol=1e-6)
    same = np.array_equal(outs[0]["power"], outs[1]["power"], equal_nan=True)
    print(f"\npk_fftpower twice: bitwise equal = {same}")
