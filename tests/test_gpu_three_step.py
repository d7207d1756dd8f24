"""GPU: three leapfrog steps per 2D launch (TPX_OPT_STEPS_2D = 3, the default).

The three-step kernel computes u^{k+1} on its tile plus a 2R halo, u^{k+2} on
the tile plus an R halo and u^{k+3} on the tile, each node with the one-step
arithmetic.  With the option set, on problems large enough for the default tile
height it takes every launch that fits a contraction block and the caller's
budget, so:
- traces, adjoint outputs and gradients are bitwise those of two-step
  launches and of one-step launches (a job advanced one step at a time);
- they match the FP64 oracle within the FP32 tolerance;
- odd block lengths and chunk sizes pair steps as 3 + 3 + 1, 3 + 2, ...
"""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built, rel_l2, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="no GPU")]

import oracle  # noqa: E402
from paper_2104_00794_amd import tpx  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d  # noqa: E402

TOL = 1e-4


@pytest.fixture(autouse=True)
def three_steps():
    ensure_built()
    old = tpx.get_option(tpx.OPT_STEPS_2D)
    tpx.set_option(tpx.OPT_STEPS_2D, 3)
    yield
    tpx.set_option(tpx.OPT_STEPS_2D, old)


def _case(order=8, nt=90, edge_sources=False, smooth_sigma=3.0):
    # 16 shots on 300 x 200 nodes: more than 512 tiles of 32 rows, so the
    # default tile height and three-step launches are chosen
    wl = small_2d(nz=200, nx=300, nt=nt, nbl=10, nshots=16, nrec=13, seed=31, order=order)
    wl = wl.with_(smooth_sigma=smooth_sigma)
    if edge_sources:
        X, Z = (wl.shape[1] - 1) * wl.h, (wl.shape[0] - 1) * wl.h
        src = list(wl.src)
        # on the physical grid's edges and corners, next to the damping layer
        src[0], src[1], src[2], src[3] = (0.0, 0.0, 0.0), (X, 0.0, Z), (0.0, 0.0, Z), (X, 0.0, 3.0)
        # on 48-column tile seams of the three-step layout (x = 48 j - 2R - nbl nodes)
        src[4] = ((48 * 3 - 10) * wl.h, 0.0, 0.4 * Z)
        src[5] = ((48 * 2 - 10 + 0.5) * wl.h, 0.0, (32 * 3 - 10 + 0.25) * wl.h)
        wl = wl.with_(src=src)
    return Case(wl)


def _uses_three_steps(c):
    # launches of a plain forward pass per kind: (three-step, two-step, one-step)
    import torch
    tpx.profile_enable(True)
    tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m0))
    torch.cuda.synchronize()
    _, n3 = tpx.profile_read(tpx.KERNEL_STEP3)
    _, n2 = tpx.profile_read(tpx.KERNEL_STEP2)
    _, n1 = tpx.profile_read(tpx.KERNEL_STEP)
    tpx.profile_enable(False)
    return n3, n2, n1


def _run_all(c, dobs, probe):
    import torch
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    out = {}
    out["d"] = to_np(tpx.forward(tg, geom, m))
    out["q"] = to_np(tpx.adjoint(tg, geom, m, d))
    g, J = tpx.gradient_probed(tg, geom, probe, m, d)
    out["g"], out["J"] = to_np(g), float(J.item())
    out["gf"] = to_np(tpx.gradient_full(tg, geom, m, d)[0])
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("order,block", [(8, 7), (8, 4), (4, 5)])
def test_three_step_launches_are_bitwise_identical(order, block):
    import torch
    ensure_built()
    print(f"[three_step] bitwise order={order} block={block}", flush=True)
    c = _case(order=order, edge_sources=True)
    dobs = c.dobs_oracle()
    probe = tpx.Probe(r=8, seed=9, block=block)
    assert tpx.get_option(tpx.OPT_STEPS_2D) == 3
    nt = c.wl.nt
    # nt - 1 = 89 steps: 29 launches of three steps and one of two
    assert _uses_three_steps(c) == (29, 1, 0) and nt == 90
    three = _run_all(c, dobs, probe)
    try:
        tpx.set_option(tpx.OPT_STEPS_2D, 2)
        assert _uses_three_steps(c) == (0, 44, 1)
        two = _run_all(c, dobs, probe)
    finally:
        tpx.set_option(tpx.OPT_STEPS_2D, 3)
    for k in three:
        assert np.array_equal(three[k], two[k]), k
    # one step per launch: a job advanced one step at a time; and odd chunks
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    for chunk in (1, 5):
        job = tpx.Job(tg, geom, probe, m, d)
        while not job.advance(chunk):
            pass
        torch.cuda.synchronize()
        assert np.array_equal(to_np(job.g), three["g"]), chunk
        assert float(job.J.item()) == three["J"], chunk


@pytest.mark.parametrize("order", [8, 4])
def test_three_step_parity_with_the_oracle(order):
    ensure_built()
    print(f"[three_step] parity order={order}", flush=True)
    # a smooth starting model and a record long enough for the residual to be
    # about 10% of the data: FP32 rounding of the traces (1e-6) then reaches the
    # gradient amplified by |d| / |d - d_obs| only about tenfold
    c = _case(order=order, nt=150, edge_sources=True, smooth_sigma=25.0)
    og = c.ogrid()
    dobs = c.dobs_oracle()
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    d_g = to_np(tpx.forward(tg, geom, cuda(c.m_true)))
    assert rel_l2(d_g, dobs) <= TOL
    q_o = oracle.adjoint(og, c.m0, c.src, c.rec, dobs)
    q_g = to_np(tpx.adjoint(tg, geom, m, d))
    assert rel_l2(q_g, q_o) <= TOL
    g_o, J_o = oracle.gradient_probed(og, c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=4)
    g_g, J_g = tpx.gradient_probed(tg, geom, tpx.Probe(r=8, seed=4), m, d)
    print("[three_step] rel", rel_l2(to_np(g_g), g_o), flush=True)
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o
    # Algorithm 1's own side: the second difference contracted in the forward pass
    g_o1, _ = oracle.gradient_probed(og, c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=4, side=1)
    g_g1, _ = tpx.gradient_probed(tg, geom, tpx.Probe(r=8, seed=4, dtt_side=1, block=10), m, d)
    assert rel_l2(to_np(g_g1), g_o1) <= TOL


def test_steps_option_is_validated():
    ensure_built()
    with pytest.raises(tpx.TpxError):
        tpx.set_option(tpx.OPT_STEPS_2D, 4)
    assert tpx.get_option(tpx.OPT_STEPS_2D) == 3


@pytest.mark.parametrize("block", [7, 16])
def test_three_steps_with_overlapped_contractions(block):
    # contractions on the auxiliary stream (ring of 2b + 3 slots) together with
    # three-step launches: the gradient is bitwise that of serial contractions
    # with two-step launches
    import torch
    print(f"[three_step] overlap block={block}", flush=True)
    c = _case(order=8, nt=90, edge_sources=True)
    dobs = c.dobs_oracle()
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=8, seed=2, block=block)
    g3, J3 = tpx.gradient_probed(tg, geom, probe, m, d)
    try:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 1)
        g3o, J3o = tpx.gradient_probed(tg, geom, probe, m, d)
        tpx.set_option(tpx.OPT_STEPS_2D, 2)
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 0)
        g2, J2 = tpx.gradient_probed(tg, geom, probe, m, d)
    finally:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 0)
        tpx.set_option(tpx.OPT_STEPS_2D, 3)
    torch.cuda.synchronize()
    assert torch.equal(g3, g3o) and torch.equal(J3, J3o)
    assert torch.equal(g3, g2) and torch.equal(J3, J2)


def test_four_remaining_steps_go_as_two_and_two():
    # contraction blocks of 7 steps: 3 + 2 + 2 (not 3 + 3 + 1); the last block
    # of each pass is 5 steps, 3 + 2.  A probed gradient then makes no one-step
    # launch, and its result is bitwise that of two-step launches.
    import torch
    print("[three_step] block remainders", flush=True)
    c = _case(order=8, nt=90)
    dobs = c.dobs_oracle()
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=8, seed=3, block=7)
    tpx.profile_enable(True)
    try:
        g3, J3 = tpx.gradient_probed(tg, geom, probe, m, d)
        torch.cuda.synchronize()
        counts = [tpx.profile_read(k)[1] for k in (tpx.KERNEL_STEP3, tpx.KERNEL_STEP2, tpx.KERNEL_STEP)]
    finally:
        tpx.profile_enable(False)
    # 89 steps per pass: twelve blocks of 7 (one three-step and two two-step
    # launches each) and one of 5 (one of each)
    assert counts == [26, 50, 0], counts
    tpx.set_option(tpx.OPT_STEPS_2D, 2)
    try:
        g2, J2 = tpx.gradient_probed(tg, geom, probe, m, d)
    finally:
        tpx.set_option(tpx.OPT_STEPS_2D, 3)
    torch.cuda.synchronize()
    assert torch.equal(g3, g2) and torch.equal(J3, J2)


def test_split_pair_and_chunked_job_match_the_gradient_call():
    # the split forward/backward pair (the autograd path) and a job advanced in
    # 64-step chunks (the serving path: 20 three-step launches and 2 + 2) give
    # the gradient call's traces, g and J bit for bit under three-step launches
    # (11-step blocks: 3 + 3 + 3 + 2)
    import torch
    print("[three_step] split pair and chunked job", flush=True)
    c = _case(order=8, nt=150)
    dobs = c.dobs_oracle()
    tg, geom, m, d = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=8, seed=5, block=11)
    g, J, d_pred = tpx.gradient_probed(tg, geom, probe, m, d, return_traces=True)
    dsp, state = tpx.forward_probed(tg, geom, probe, m)
    g_split = tpx.backward_probed(tg, geom, probe, m, dsp - d, state)
    job = tpx.Job(tg, geom, probe, m, d)
    while not job.advance(64):
        pass
    torch.cuda.synchronize()
    assert torch.equal(dsp, d_pred)
    assert torch.equal(g_split, g)
    assert torch.equal(job.g, g) and torch.equal(job.J, J)


@pytest.mark.parametrize("nx,nz,shots,tile", [(140, 60, 4, 8), (300, 120, 14, 16)])
def test_three_steps_on_short_tiles(nx, nz, shots, tile):
    # small problems take 8- or 16-row tiles; their three-step launches use the
    # same tile height: traces, the adjoint, the probed and the full-storage
    # gradient are bitwise those of two-step launches (the oracle parity of
    # small problems is checked by the parity tests, which run three-step
    # launches by default)
    import torch
    print(f"[three_step] short tiles {nx}x{nz} shots={shots}", flush=True)
    wl = small_2d(nz=nz, nx=nx, nt=120, nbl=10, nshots=shots, nrec=11, seed=17)
    c = Case(wl.with_(smooth_sigma=15.0))
    dobs = c.dobs_oracle()
    probe = tpx.Probe(r=8, seed=2, block=10)
    n3 = _uses_three_steps(c)
    assert n3[0] > 0 and n3[2] == 0, n3
    three = _run_all(c, dobs, probe)
    try:
        tpx.set_option(tpx.OPT_STEPS_2D, 2)
        assert _uses_three_steps(c)[0] == 0
        two = _run_all(c, dobs, probe)
    finally:
        tpx.set_option(tpx.OPT_STEPS_2D, 3)
    for k in three:
        assert np.array_equal(three[k], two[k]), k
