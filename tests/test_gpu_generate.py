"""GPU parity of the device Gaussian-field generator (pk_fft_r2c,
pk_shape_spectrum, pk_fft_c2r; Sec. 3.2 catalogs from Gaussian fields):
with the same white noise it reproduces the host recipe of the input
generator (SciPy float64 transforms), and the shaping alone matches the
oracle's transform of the shaped spectrum.  Tolerances relative to the rms:
float64 1e-12, float32 1e-6 (rms) and 1e-4 (max)."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, generate, synth
from tests import packing

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def rel(got, want):
    rms = math.sqrt(np.mean(want ** 2))
    return (math.sqrt(np.mean((got - want) ** 2)) / rms, np.abs(got - want).max() / rms)


@pytest.mark.parametrize("dtype", ["f8", "f4"])
@pytest.mark.parametrize("n", [32, 128])
def test_device_gaussian_field_matches_the_host_recipe(ctx, dtype, n):
    box, seed = 500.0, 9
    want = synth.gaussian_field(n, box, synth.pk_lognormal_c2, seed)
    noise = synth.rng_for(seed).standard_normal((n, n, n))  # the recipe's own draws
    tdt = torch.float64 if dtype == "f8" else torch.float32
    got = generate.gaussian_field(ctx, torch.from_numpy(noise).to("cuda:0", tdt), box,
                                  synth.pk_lognormal_c2)
    er, em = rel(got.double().cpu().numpy(), want)
    print(f"n={n} {dtype}: rms {er:.2e} max {em:.2e}")
    tol = (1e-12, 1e-11) if dtype == "f8" else (1e-6, 1e-4)
    assert er <= tol[0] and em <= tol[1], (er, em)


@pytest.mark.parametrize("n", [16, 64])
def test_shaping_matches_oracle_on_the_packed_layout(ctx, n):
    rng = np.random.default_rng(n)
    c = oracle.r2c(rng.standard_normal((n, n, n)))
    table = rng.uniform(0.5, 2.0, _lib.shape_table_len(_lib.mesh_desc(n, 1.0)))
    nx, ny, nz = oracle.mode_indices(n)
    n2 = nx[:, None, None] ** 2 + ny[None, :, None] ** 2 + nz[None, None, :] ** 2
    want = packing.pack(c * table[n2])
    m = _lib.mesh_desc(n, 1.0, "cic", False, False, "f8")
    mesh = torch.from_numpy(packing.to_real_view(packing.pack(c), np.float64)).to("cuda:0")
    ctx.pk_shape_spectrum(m, mesh, torch.from_numpy(table).to("cuda:0"))
    got = packing.as_complex(mesh.cpu().numpy())
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
