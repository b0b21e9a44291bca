"""Run-time tuning of pk_fftpower's launch choices: every choice the tuner
can make (two-mesh or split painting of interlaced meshes, x-pass
workgroups per CU) gives the result of the default settings bit for bit, for
every window; a tuned context and a context loaded with its table give that
result too.  (The painting's cell sums and the bin sums are exact
fixed-point sums, so the tiling and the number of workgroups do not change
a bit.)"""

import itertools

import numpy as np
import pytest
import torch

from paper_1712_05834_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _run(ctx, m, b, pos, ws):
    r = torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")
    ctx.pk_fftpower(m, b, pos, None, pos.shape[0], ws, r)
    return ctx.pk_result_to_host(m, b, r)


def _same(a, b, tag):
    for key in ("modes", "k", "power", "power2d", "shotnoise"):
        if key in b:
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{tag} {key}")
    for ell in b["poles"]:
        np.testing.assert_array_equal(a["poles"][ell], b["poles"][ell], err_msg=f"{tag} P_{ell}")


@pytest.mark.parametrize("window", ["cic", "tsc", "pcs"])
def test_every_tuning_choice_gives_the_default_result(window):
    n, box = 64, 400.0
    pos = torch.from_numpy(synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 1.0, seed=31)
                           ).to("cuda:0")
    npart = pos.shape[0]
    m = _lib.mesh_desc(n, box, window, True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 3, (0, 2, 4), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, npart), dtype=torch.uint8, device="cuda:0")
    ref_ctx = _lib.Context(0)
    want = _run(ref_ctx, m, b, pos, ws)
    ctx = _lib.Context(0)
    dens = int(round(np.log2(npart / n ** 3)))
    for split, xpc in itertools.product((0, 1), (0, 1, 2)):
        ctx.tune_load([{"nmesh": n, "dtype": 0, "window": m.window, "interlaced": 1,
                        "density": dens, "split": split, "xpass_per_cu": xpc, "ms": 0.0}])
        _same(_run(ctx, m, b, pos, ws), want, f"{window} split={split} xpc={xpc}")
    ctx.close()
    ref_ctx.close()


def test_autotune_picks_and_reuses_a_choice():
    n, box = 128, 700.0
    pos = torch.from_numpy(synth.uniform_catalog(400_000, box, seed=32).astype(np.float32)
                           ).to("cuda:0")
    m = _lib.mesh_desc(n, box, "tsc", True, True, "f4")
    b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2), 2)
    ws = torch.empty(_lib.workspace_bytes(m, b, 400_000), dtype=torch.uint8, device="cuda:0")
    ctx = _lib.Context(0)
    want = _run(ctx, m, b, pos, ws)  # defaults (tuning off)
    ctx.pk_ctx_set_autotune(1)
    got = _run(ctx, m, b, pos, ws)   # tunes on this call
    table = ctx.tune_table()
    assert len(table) == 1
    e = table[0]
    assert (e["nmesh"], e["window"], e["interlaced"]) == (128, 3, 1)
    assert e["split"] in (0, 1) and e["xpass_per_cu"] in (0, 1)
    assert e["ms"] > 0
    print(f"\ntuned 128^3 TSC interlaced, 400k particles: {e}")
    _same(got, want, "tuned call")
    _same(_run(ctx, m, b, pos, ws), want, "second call")
    assert len(ctx.tune_table()) == 1  # no new tuning for the same key
    other = _lib.Context(0)
    other.tune_load(table)
    _same(_run(other, m, b, pos, ws), want, "loaded table")
    other.close()
    ctx.close()
