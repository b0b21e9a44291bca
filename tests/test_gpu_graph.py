"""Graph-captured batches (pk_fftpower_batch_graph, pk_graph_launch): every
replay of the captured batch against the same batch run eagerly, with eager
work and synchronisations between the replays; a replay after the positions
were overwritten in place against the eager result of the new positions; and
a capture on a context without lanes.

The painting's cell sums and the bin sums are exact fixed-point sums and the
FFT passes are deterministic, so replays and eager runs agree bit for bit."""

import numpy as np
import pytest
import torch

from paper_1712_05834_amd import _lib, synth

pytestmark = pytest.mark.gpu

MESHES = (32, 64, 128, 64, 32, 128)


def _batch(seed):
    rng = np.random.default_rng(seed)
    pos, ms, bs = [], [], []
    for i, n in enumerate(MESHES):
        box = 500.0
        if i % 2:
            p = synth.lognormal_catalog(n, box, synth.pk_lognormal_c2, 0.3, seed=seed + i)
        else:
            p = rng.uniform(0, box, (int(rng.integers(1000, 60000)), 3)).astype(np.float32)
        pos.append(torch.from_numpy(np.ascontiguousarray(p)).to("cuda:0"))
        ms.append(_lib.mesh_desc(n, box, "tsc" if i % 3 else "cic", bool(i % 2 == 0), True, "f4"))
        bs.append(_lib.bin_desc(n // 2, 0.0, 1.0, 4 if i % 2 else 0, (0, 2, 4), 2))
    return pos, ms, bs


def _workspaces(ms, bs, pos, lanes):
    need = max(_lib.workspace_bytes(m, b, p.shape[0]) for m, b, p in zip(ms, bs, pos))
    return [torch.empty(need, dtype=torch.uint8, device="cuda:0") for _ in range(max(lanes, 1))]


def _results(bs):
    return [torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0") for b in bs]


def _host(ctx, ms, bs, res):
    return [ctx.pk_result_to_host(m, b, r) for m, b, r in zip(ms, bs, res)]


def _same(a, b, tag):
    for key in ("modes", "k", "power", "modes2d", "power2d", "shotnoise"):
        if key in b:
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{tag} {key}")
    for ell in b["poles"]:
        np.testing.assert_array_equal(a["poles"][ell], b["poles"][ell], err_msg=f"{tag} P_{ell}")


@pytest.mark.parametrize("lanes", [3, 0])
def test_graph_replays_match_the_eager_batch(lanes):
    stream = torch.cuda.Stream(device="cuda:0")
    ctx = _lib.Context(0, stream)
    if lanes:
        ctx.pk_ctx_set_lanes(lanes)
    pos, ms, bs = _batch(seed=100 + lanes)
    n = [p.shape[0] for p in pos]
    ws = _workspaces(ms, bs, pos, lanes)
    eager_res = _results(bs)
    with torch.cuda.stream(stream):
        if lanes:
            ctx.pk_fftpower_batch(ms, bs, pos, [None] * len(pos), n, ws, eager_res)
        else:
            for i in range(len(pos)):
                ctx.pk_fftpower(ms[i], bs[i], pos[i], None, n[i], ws[0], eager_res[i])
        want = _host(ctx, ms, bs, eager_res)
        graph_res = _results(bs)
        graph = ctx.pk_fftpower_batch_graph(ms, bs, pos, [None] * len(pos), n, ws, graph_res)
        assert graph.nodes >= 5 * len(pos)
        other = torch.from_numpy(synth.uniform_catalog(5000, 300.0, seed=9).astype(np.float32))
        other = other.to("cuda:0")
        m_o = _lib.mesh_desc(64, 300.0, "pcs", True, True, "f4")
        b_o = _lib.bin_desc(32, 0.0, 1.0, 0, (0, 2), 2)
        ws_o = torch.empty(_lib.workspace_bytes(m_o, b_o, 5000), dtype=torch.uint8,
                           device="cuda:0")
        r_o = torch.empty(_lib.result_doubles(b_o), dtype=torch.float64, device="cuda:0")
        for rep in range(3):
            for r in graph_res:
                r.fill_(float("nan"))
            graph.launch()
            got = _host(ctx, ms, bs, graph_res)
            for i in range(len(pos)):
                _same(got[i], want[i], f"replay {rep}, request {i}")
            # eager work and a synchronisation between replays
            ctx.pk_fftpower(m_o, b_o, other, None, 5000, ws_o, r_o)
            ctx.pk_result_to_host(m_o, b_o, r_o)
            torch.cuda.synchronize()
        # positions overwritten in place: the replay reads the new ones
        fresh = synth.uniform_catalog(n[0], 500.0, seed=77).astype(np.float32)
        pos[0].copy_(torch.from_numpy(fresh))
        graph.launch()
        got0 = _host(ctx, ms[:1], bs[:1], graph_res[:1])[0]
        ctx.pk_fftpower(ms[0], bs[0], pos[0], None, n[0], ws[0], eager_res[0])
        want0 = _host(ctx, ms[:1], bs[:1], eager_res[:1])[0]
        _same(got0, want0, "replay after new positions")
        graph.close()
    torch.cuda.synchronize()
    ctx.close()


def test_graph_capture_refuses_timing_and_empty_batches():
    stream = torch.cuda.Stream(device="cuda:0")
    ctx = _lib.Context(0, stream)
    pos, ms, bs = _batch(seed=5)
    n = [p.shape[0] for p in pos]
    ws = _workspaces(ms, bs, pos, 0)
    with pytest.raises(_lib.PkError):
        ctx.pk_fftpower_batch_graph([], [], [], [], [], ws, [])
    ctx.pk_ctx_set_timing(True)
    with pytest.raises(_lib.PkError):
        ctx.pk_fftpower_batch_graph(ms, bs, pos, [None] * len(pos), n, ws, _results(bs))
    ctx.pk_ctx_set_timing(False)
    ctx.close()
