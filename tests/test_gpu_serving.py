"""Serving: continuous batching of probed-gradient jobs on one GPU."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import ensure_built

pytestmark = pytest.mark.gpu

if gpu_available():
    ensure_built()

import torch  # noqa: E402

from paper_2104_00794_amd import serve, tpx  # noqa: E402
from paper_2104_00794_amd.inputs import serving_workload  # noqa: E402


def make_request(i, seed=41, small=True, arrival=0.0):
    wl = serving_workload(i, seed, small=small)
    mt, m0 = wl.models()
    dev = torch.device("cuda")
    grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
    geom = tpx.Geometry(wl.src_pos(), wl.rec_pos(), torch.tensor(wl.wavelet(), dtype=torch.float32, device=dev))
    probe = tpx.Probe(r=wl.r, seed=wl.probe_seed)
    d_obs = tpx.forward(grid, geom, torch.tensor(mt, dtype=torch.float32, device=dev))
    m = torch.tensor(m0, dtype=torch.float32, device=dev)
    return serve.Request(i, grid, geom, probe, m, d_obs, arrival)


def test_job_in_chunks_equals_one_call():
    req = make_request(3)
    g, J = tpx.gradient_probed(req.grid, req.geom, req.probe, req.m, req.d_obs)
    job = tpx.Job(req.grid, req.geom, req.probe, req.m, req.d_obs)
    n = 0
    while not job.advance(7):
        n += 1
    torch.cuda.synchronize()
    assert n > 2
    assert torch.equal(job.g, g) and torch.equal(job.J, J)
    done, total = job.progress()
    assert done == total == 2 * (req.grid.nt - 1)


def test_results_identical_alone_and_in_the_mix():
    reqs = [make_request(i, arrival=0.002 * i) for i in range(10)]
    alone = serve.run_sequential(reqs)
    srv = serve.Server(hbm_budget_bytes=50e9, chunk_steps=32, max_active=8, nstreams=6)
    mixed = srv.run(reqs)
    assert srv.peak_active > 1
    for r in reqs:
        a, b = alone[r.rid], mixed[r.rid]
        assert b.status == "ok"
        assert torch.equal(a.g, b.g), r.rid
        assert torch.equal(a.J, b.J), r.rid
    s = serve.summarize(mixed, reqs)
    assert s["completed"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_one_large_job_at_a_time():
    # with the large-job threshold at the median job size, at most one large
    # job runs while small ones pass it; results stay bitwise those of the
    # plain path
    reqs = [make_request(i) for i in range(10)]
    sizes = sorted(q.geom.nshots * int(np.prod([n + 2 * q.grid.nbl for n in q.grid.shape])) for q in reqs)
    alone = serve.run_sequential(reqs)
    srv = serve.Server(hbm_budget_bytes=50e9, chunk_steps=32, max_active=4, nstreams=6,
                       large_points=sizes[len(sizes) // 2], max_large=1)
    mixed = srv.run(reqs)
    assert srv.peak_large == 1 and srv.peak_active > 1
    for r in reqs:
        assert mixed[r.rid].status == "ok"
        assert torch.equal(alone[r.rid].g, mixed[r.rid].g), r.rid


def test_admission_by_hbm_budget():
    reqs = [make_request(i, arrival=0.0) for i in range(4)]
    need = [r.workspace_bytes() for r in reqs]
    budget = max(need) * 1.05 + 1e6     # room for one job at a time (the largest)
    srv = serve.Server(hbm_budget_bytes=budget, chunk_steps=64, max_active=4, nstreams=4)
    res = srv.run(reqs)
    assert all(r.status == "ok" for r in res.values())
    assert srv.peak_bytes <= budget
    tiny = serve.Server(hbm_budget_bytes=min(need) / 2, chunk_steps=64)
    res = tiny.run(reqs[:2])
    assert all(r.status.startswith("rejected") for r in res.values())


def test_cancellation_frees_the_workspace_and_leaves_the_others_unchanged():
    reqs = [make_request(i, arrival=0.0) for i in range(6)]
    alone = serve.run_sequential(reqs)
    reqs[1].cancel_at = 0.0          # withdrawn before it can start
    reqs[2].cancel_at = 0.01         # withdrawn while running (or waiting)
    srv = serve.Server(hbm_budget_bytes=50e9, chunk_steps=16, max_active=3, nstreams=4)
    res = srv.run(reqs)
    assert res[1].status == "cancelled" and res[1].g is None
    assert res[2].status in ("cancelled", "ok")
    assert srv.in_use_bytes == 0
    for r in reqs:
        if r.rid in (1, 2):
            continue
        assert res[r.rid].status == "ok"
        assert torch.equal(res[r.rid].g, alone[r.rid].g) and torch.equal(res[r.rid].J, alone[r.rid].J)
    s = serve.summarize(res, reqs)
    assert s["cancelled"] >= 1 and s["completed"] + s["cancelled"] == len(reqs)
