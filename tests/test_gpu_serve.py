"""Serving: every request served in a concurrent mix gives the result it
gives alone (within the float32 bar), and the oracle's.

Twelve requests of mixed mesh sizes, windows, interlacing, catalog kinds and
sizes arrive in a burst, so that four lanes run them concurrently."""

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, synth
from paper_1712_05834_amd.serve import LibpkBackend, Request, Server, latency_stats
from tests.powercheck import check_power

pytestmark = pytest.mark.gpu


def build_requests():
    rng = np.random.default_rng(55)
    reqs = []
    for i in range(12):
        n = [32, 64, 128][i % 3]
        box = float(rng.uniform(200, 1500))
        window = ["cic", "tsc", "pcs"][(i // 3) % 3]
        inter = bool(i % 2)
        npart = int(10 ** rng.uniform(3, 5.3))
        if i % 4 == 3:
            pos = synth.lognormal_catalog_device(n, box, synth.pk_lognormal_c2, npart / n ** 3,
                                                 seed=500 + i, device="cuda:0")
        else:
            pos = torch.from_numpy(synth.uniform_catalog(npart, box, seed=500 + i,
                                                         dtype=np.float32)).to("cuda:0")
        m = _lib.mesh_desc(n, box, window, inter, True, "f4")
        b = _lib.bin_desc(n // 2, 0.0, 1.0, 3 if i % 3 == 0 else 0, (0, 2), 2)
        reqs.append(Request(i, 0.0005 * i, m, b, pos, pos.shape[0]))
    return reqs


def test_same_alone_and_in_the_mix():
    ctx = _lib.Context(0)
    backend = LibpkBackend(ctx, lanes=4)
    reqs = build_requests()
    print(f"\nserving {len(reqs)} requests on 4 lanes", flush=True)
    served = Server(backend, budget=16 << 30).run(reqs)
    st = latency_stats(served)
    print(f"p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms", flush=True)
    assert len({r.lane for r in served}) > 1, "the burst should use several lanes"
    for r in served:
        ws = torch.empty(_lib.workspace_bytes(r.mesh, r.bins, r.npart), dtype=torch.uint8,
                         device="cuda:0")
        res = torch.empty(_lib.result_doubles(r.bins), dtype=torch.float64, device="cuda:0")
        ctx.pk_fftpower(r.mesh, r.bins, r.pos, None, r.npart, ws, res)
        alone = ctx.pk_result_to_host(r.mesh, r.bins, res)
        check_power(r.result, alone, 1e-5, f"request {r.rid} mix vs alone")
    for r in served[:3]:
        want = oracle.fftpower(r.pos.cpu().numpy().astype(np.float64), r.mesh.nmesh,
                               r.mesh.boxsize, int(r.mesh.window), bool(r.mesh.interlaced), True,
                               nk=r.bins.nk, nmu=r.bins.nmu, poles=(0, 2))
        check_power(r.result, want, 1e-5, f"request {r.rid} vs oracle")
    torch.cuda.synchronize()
    ctx.close()
