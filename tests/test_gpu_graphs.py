"""The gradient call captured into a HIP graph (torch.cuda.graph) and
replayed: every replay equals the eager call bit for bit, with eager library
work and synchronisations between the replays."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built

pytestmark = pytest.mark.gpu

if gpu_available():
    ensure_built()

from paper_2104_00794_amd import tpx  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d, small_3d  # noqa: E402


@pytest.mark.parametrize("ndim,r", [(2, 8), (2, 64), (3, 32)])
def test_captured_gradient_replays_bitwise(ndim, r):
    import torch
    print("[case] graph", ndim, r, flush=True)
    c = Case(small_2d(nz=40, nx=150, nt=220, nshots=3, nrec=17) if ndim == 2 else
             small_3d(nz=40, ny=11, nx=70, nt=90, nshots=2, nrec=9))
    m, d = cuda(c.m0), cuda(c.dobs_oracle())
    grid, geom = c.tgrid(), c.tgeom()
    probe = tpx.Probe(r=r, seed=17, block=37)
    g_ref, J_ref = tpx.gradient_probed(grid, geom, probe, m, d)
    ws = tpx.alloc_workspace(tpx.CALL_GRADIENT_PROBED, grid, geom, probe)
    g = torch.empty_like(g_ref)
    J = torch.empty_like(J_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up on the capture stream
        tpx.gradient_probed(grid, geom, probe, m, d, ws=ws, g_out=g, J_out=J)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s, capture_error_mode="relaxed"):
        tpx.gradient_probed(grid, geom, probe, m, d, ws=ws, g_out=g, J_out=J)
    for i in range(4):
        g.fill_(float("nan"))
        J.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref) and torch.equal(J, J_ref), i
        # eager library work in between, on the same workspace-free path
        tpx.forward(grid, geom, m)
        torch.cuda.synchronize()
    assert np.isfinite(g.cpu().numpy()).all()
