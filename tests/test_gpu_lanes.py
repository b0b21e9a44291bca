"""Lanes and batches (concurrent requests on one GPU): every request run on
a lane or inside a batch gives the result it gives alone, and the oracle's.

A batch mixes mesh sizes, windows, interlacing, precisions, weights and
binnings; a lane request is checked while other lanes run."""

import numpy as np
import pytest
import torch

import oracle
from paper_1712_05834_amd import _lib, synth
from tests.powercheck import check_power

pytestmark = pytest.mark.gpu

TOL = {"f8": 1e-12, "f4": 1e-5}
TDT = {"f8": torch.float64, "f4": torch.float32}
NDT = {"f8": np.float64, "f4": np.float32}

# (n, box, window, interlaced, dtype, npart, weighted, nk, nmu, poles, seed)
REQUESTS = [
    (64, 500.0, "tsc", True, "f4", 40000, False, 32, 5, (0, 2, 4), 11),
    (32, 300.0, "cic", False, "f8", 5000, True, 16, 0, (), 12),
    (128, 1380.0, "pcs", True, "f4", 150000, False, 64, 0, (0, 2), 13),
    (64, 800.0, "cic", True, "f8", 20000, False, 32, 3, (2,), 14),
    (16, 100.0, "tsc", False, "f4", 0, False, 8, 0, (), 15),     # empty catalog
    (32, 250.0, "pcs", False, "f4", 3000, True, 24, 4, (0, 4), 16),
    (64, 600.0, "tsc", True, "f4", 1, False, 32, 0, (0,), 17),    # one particle
]


@pytest.fixture(scope="module")
def ctx():
    c = _lib.Context(0)
    c.pk_ctx_set_lanes(3)
    yield c
    torch.cuda.synchronize()
    c.close()


def make(req):
    n, box, window, inter, dt, npart, weighted, nk, nmu, poles, seed = req
    pos = synth.uniform_catalog(npart, box, seed=seed, dtype=NDT[dt])
    w = synth.uniform_weights(npart, seed=seed + 1).astype(NDT[dt]) if weighted else None
    m = _lib.mesh_desc(n, box, window, inter, True, dt)
    b = _lib.bin_desc(nk, 0.0, 1.0, nmu, poles, 2)
    d = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return dict(pos=pos, w=w, m=m, b=b, dpos=d(pos) if npart else torch.empty((0, 3), dtype=TDT[dt], device="cuda:0"),
                dw=d(w), res=torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0"))


def oracle_of(req, r):
    n, box, window, inter, dt, npart, weighted, nk, nmu, poles, seed = req
    return oracle.fftpower(r["pos"].astype(np.float64), n, box, window, inter, True,
                           None if r["w"] is None else r["w"].astype(np.float64),
                           nk=nk, nmu=nmu, poles=poles)


def compare(got, want, tol, tag, npart):
    if npart == 0:
        # an empty catalog: sum w = 0, so no power is defined; counts still exact
        np.testing.assert_array_equal(got["modes"], want["modes"], err_msg=tag)
        assert not np.any(np.isfinite(got["power"])), tag
        return
    check_power(got, want, tol, tag)


def test_batch_matches_alone_and_oracle(ctx):
    reqs = [make(q) for q in REQUESTS]
    m0 = max(_lib.workspace_bytes(r["m"], r["b"], max(q[5], 1)) for q, r in zip(REQUESTS, reqs))
    lane_ws = [torch.empty(m0, dtype=torch.uint8, device="cuda:0") for _ in range(3)]
    print(f"\nbatch of {len(reqs)} requests on 3 lanes", flush=True)
    ctx.pk_fftpower_batch([r["m"] for r in reqs], [r["b"] for r in reqs], [r["dpos"] for r in reqs],
                          [r["dw"] for r in reqs], [q[5] for q in REQUESTS], lane_ws,
                          [r["res"] for r in reqs])
    batch = [ctx.pk_result_to_host(r["m"], r["b"], r["res"]) for r in reqs]
    for q, r, got in zip(REQUESTS, reqs, batch):
        tag = f"n{q[0]} {q[2]} inter={q[3]} {q[4]} np={q[5]}"
        ws = torch.empty(_lib.workspace_bytes(r["m"], r["b"], q[5]), dtype=torch.uint8,
                         device="cuda:0")
        res = torch.empty_like(r["res"])
        ctx.pk_fftpower(r["m"], r["b"], r["dpos"], r["dw"], q[5], ws, res)
        alone = ctx.pk_result_to_host(r["m"], r["b"], res)
        compare(got, alone, TOL[q[4]], tag + " batch vs alone", q[5])
        if q[5] > 0:  # the oracle's P is undefined for an empty catalog (sum w = 0)
            compare(got, oracle_of(q, r), TOL[q[4]], tag + " batch vs oracle", q[5])


def test_async_lanes_while_others_run(ctx):
    big = make((128, 1380.0, "tsc", True, "f4", 400000, False, 64, 5, (0, 2, 4), 21))
    small = make(REQUESTS[1])
    wsb = torch.empty(_lib.workspace_bytes(big["m"], big["b"], 400000), dtype=torch.uint8,
                      device="cuda:0")
    wss = torch.empty(_lib.workspace_bytes(small["m"], small["b"], REQUESTS[1][5]),
                      dtype=torch.uint8, device="cuda:0")
    # the big request twice on lane 0, the small one on lane 2 in between
    ctx.pk_fftpower_async(0, big["m"], big["b"], big["dpos"], None, 400000, wsb, big["res"])
    ctx.pk_fftpower_async(2, small["m"], small["b"], small["dpos"], small["dw"], REQUESTS[1][5],
                          wss, small["res"])
    ctx.pk_lane_wait(2)
    assert ctx.pk_lane_query(2)
    got_small = ctx.pk_result_to_host(small["m"], small["b"], small["res"])
    ctx.pk_lane_wait(0)
    assert ctx.pk_lane_query(0)
    got_big = ctx.pk_result_to_host(big["m"], big["b"], big["res"])
    compare(got_small, oracle_of(REQUESTS[1], small), TOL["f8"], "small lane", REQUESTS[1][5])
    want_big = oracle.fftpower(big["pos"].astype(np.float64), 128, 1380.0, "tsc", True, True,
                               nk=64, nmu=5, poles=(0, 2, 4))
    compare(got_big, want_big, TOL["f4"], "big lane", 400000)


def test_device_lognormal_mocks_match_oracle(ctx):
    """A small batch shaped like the many-mock workload: device-drawn
    log-normal catalogs, TSC interlaced, P(k) with ell = 0, 2, 4."""
    sizes = [(30000, 32), (120000, 64), (60000, 32), (200000, 64)]
    reqs = []
    for i, (npart, n) in enumerate(sizes):
        pos = synth.lognormal_catalog_device(n, 1380.0, synth.pk_lognormal_c2, npart / n ** 3,
                                             seed=1000 + i, device="cuda:0")
        m = _lib.mesh_desc(n, 1380.0, "tsc", True, True, "f4")
        b = _lib.bin_desc(n // 2, 0.0, 1.0, 0, (0, 2, 4), 2)
        reqs.append(dict(m=m, b=b, dpos=pos, n=pos.shape[0],
                         res=torch.empty(_lib.result_doubles(b), dtype=torch.float64, device="cuda:0")))
    m0 = max(_lib.workspace_bytes(r["m"], r["b"], r["n"]) for r in reqs)
    lane_ws = [torch.empty(m0, dtype=torch.uint8, device="cuda:0") for _ in range(3)]
    ctx.pk_fftpower_batch([r["m"] for r in reqs], [r["b"] for r in reqs], [r["dpos"] for r in reqs],
                          [None] * len(reqs), [r["n"] for r in reqs], lane_ws, [r["res"] for r in reqs])
    for (npart, n), r in zip(sizes, reqs):
        got = ctx.pk_result_to_host(r["m"], r["b"], r["res"])
        want = oracle.fftpower(r["dpos"].cpu().numpy().astype(np.float64), n, 1380.0, "tsc", True,
                               True, nk=n // 2, poles=(0, 2, 4))
        check_power(got, want, TOL["f4"], f"mock n{n} np{r['n']}")
