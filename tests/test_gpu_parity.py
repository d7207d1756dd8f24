"""GPU parity: the HIP library against the FP64 oracle on identical seeded
inputs.  Bars: probes bit-exact; traces, adjoint outputs and gradients within
relative L2 <= 1e-4 (FP32 on the GPU vs FP64 in the oracle).

Sizes span several step-kernel tiles (64 x 16 in 2D, 64 x 8 columns with
12-plane z chunks in 3D) with ragged edges, both stencil orders, several
shots, off-grid and on-grid sources/receivers, and the edge cases nt = 2,
no receivers, receivers on the last grid line.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-4

if gpu_available():
    ensure_built()

import oracle  # noqa: E402
from paper_2104_00794_amd import tpx  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d, small_3d, workload  # noqa: E402


def _print_case(name, **kw):
    print("[case]", name, kw, flush=True)


# --------------------------------------------------------------------------- #
# probes
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("kind", ["rademacher", "gauss_b64"])
def test_probe_matrix_bit_exact(kind):
    for seed, shot, nt, r in ((0, 0, 37, 5), (12, 7, 2401, 64), (2 ** 63 + 11, 3, 129, 32)):
        _print_case("probe", kind=kind, seed=seed, shot=shot, nt=nt, r=r)
        Zg = to_np(tpx.probe_matrix(tpx.Probe(kind=kind, r=r, seed=seed), nt, shot))
        Zo = oracle.probe_matrix(kind, r, seed, nt, shot)
        assert np.array_equal(Zg, Zo)


def test_identity_probe_matrix():
    Zg = to_np(tpx.probe_matrix(tpx.Probe(kind="identity", r=33), 33, 0))
    assert np.array_equal(Zg, np.eye(33))


# --------------------------------------------------------------------------- #
# forward and adjoint
# --------------------------------------------------------------------------- #

CASES_2D = [
    dict(nz=40, nx=150, order=8, nt=200, nbl=6, nshots=3, nrec=17),   # several x tiles, ragged
    dict(nz=37, nx=29, order=4, nt=160, nbl=9, nshots=2, nrec=5),     # ragged in x and z
]


@pytest.mark.parametrize("kw", CASES_2D)
def test_forward_traces_2d(kw):
    _print_case("forward2d", **kw)
    c = Case(small_2d(**kw))
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, d_o) <= TOL


def test_forward_traces_3d():
    kw = dict(nz=40, ny=11, nx=70, nt=90, nbl=5, nshots=2, nrec=9)   # 2 z-chunks, ragged y/x tiles
    _print_case("forward3d", **kw)
    c = Case(small_3d(**kw))
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, d_o) <= TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_matches_oracle_and_dot_test(ndim):
    _print_case("adjoint", ndim=ndim)
    c = Case(small_2d(nz=33, nx=70, nt=150) if ndim == 2 else small_3d(nt=70, nshots=2))
    rng = np.random.default_rng(4)
    d_in = rng.normal(size=(c.wl.nshots, c.wl.nt, c.rec.shape[1])).astype(np.float32).astype(np.float64)
    q_o = oracle.adjoint(c.ogrid(), c.m_true, c.src, c.rec, d_in)
    q_g = to_np(tpx.adjoint(c.tgrid(), c.tgeom(), cuda(c.m_true), cuda(d_in)))
    assert rel_l2(q_g, q_o) <= TOL
    # dot test on the GPU path alone
    q = rng.normal(size=(c.wl.nshots, c.wl.nt)).astype(np.float32)
    geom = tpx.Geometry(c.src, c.rec, cuda(q))
    Fq = to_np(tpx.forward(c.tgrid(), geom, cuda(c.m_true)))
    lhs, rhs = np.sum(Fq * d_in), np.sum(q.astype(np.float64) * q_g)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_edge_cases_forward():
    # nt = 2; receivers exactly on the last grid line and corner; one shot
    wl = small_2d(nz=20, nx=21, nt=2, nshots=1, nrec=3)
    X, Zd = (wl.shape[1] - 1) * wl.h, (wl.shape[0] - 1) * wl.h
    wl = wl.with_(rec=[(X, 0.0, Zd), (0.0, 0.0, 0.0), (X / 2, 0.0, Zd)])
    c = Case(wl)
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert np.all(d_o[:, 0] == 0) and np.all(d_g[:, 0] == 0)
    np.testing.assert_allclose(d_g, d_o, rtol=0, atol=1e-6 * max(np.abs(d_o).max(), 1e-30))
    # longer record with the same edge receivers
    c = Case(wl.with_(nt=120))
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, d_o) <= TOL


def test_no_receivers_gradient_is_zero():
    wl = small_2d(nt=80).with_(rec=[])
    c = Case(wl)
    zero = np.zeros((wl.nshots, wl.nt, 0))
    g, J = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=4, seed=1), cuda(c.m0), cuda(zero))
    assert float(J.item()) == 0.0
    assert np.all(to_np(g) == 0.0)


# --------------------------------------------------------------------------- #
# gradients
# --------------------------------------------------------------------------- #

def _grad_case(ndim):
    if ndim == 2:
        return Case(small_2d(nz=40, nx=150, nt=220, nshots=3, nrec=17))
    return Case(small_3d(nz=40, ny=11, nx=70, nt=90, nshots=2, nrec=9))


@pytest.mark.parametrize("ndim", [2, 3])
def test_full_gradient_matches_oracle(ndim):
    _print_case("grad_full", ndim=ndim)
    c = _grad_case(ndim)
    dobs = c.dobs_oracle()
    g_o, J_o = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_g, J_g, d_g = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs), return_traces=True)
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("kind", ["rademacher", "gauss_b64"])
@pytest.mark.parametrize("keep_vbar", [False, True])
def test_probed_gradient_matches_oracle(ndim, kind, keep_vbar):
    _print_case("grad_probed", ndim=ndim, kind=kind, keep_vbar=keep_vbar)
    c = _grad_case(ndim)
    dobs = c.dobs_oracle()
    r, seed = 6, 77
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind=kind, r=r, seed=seed)
    probe = tpx.Probe(kind=kind, r=r, seed=seed, block=13, keep_vbar=keep_vbar)  # ragged time blocks
    g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("r", [16, 64, 70])
def test_probed_gradient_probe_counts(r):
    # register-chunk boundaries of the contraction kernels (8/16/32/64 and beyond)
    _print_case("grad_probed_r", r=r)
    c = Case(small_2d(nz=30, nx=90, nt=150, nshots=2, nrec=11))
    dobs = c.dobs_oracle()
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=5)
    g_g, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=r, seed=5), cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL


@pytest.mark.parametrize("ndim,r,block,mfma", [(2, 1, 1, 1), (2, 3, 149, 1), (2, 5, 2, 1), (2, 16, 1, 2),
                                               (2, 32, 3, 2), (3, 1, 1, 1), (3, 16, 2, 2), (2, 160, 0, 1),
                                               (2, 150, 0, 1), (3, 96, 0, 1)])
def test_probed_gradient_degenerate_blocks(ndim, r, block, mfma):
    # one probe; one buffered level per contraction block (a 3-slot ring);
    # one block for the whole record; 16-level matrix-core tiles holding 1-3
    # live levels; more probes than time samples (r > nt)
    _print_case("grad_blocks", ndim=ndim, r=r, block=block, mfma=mfma)
    c = Case(small_2d(nz=30, nx=90, nt=150, nshots=2, nrec=11) if ndim == 2 else
             small_3d(nz=20, ny=12, nx=30, nt=60, nshots=2, nrec=7))
    dobs = c.dobs_oracle()
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=21)
    old = tpx.get_option(tpx.OPT_MATRIX_CORES)
    try:
        tpx.set_option(tpx.OPT_MATRIX_CORES, mfma)
        g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=r, seed=21, block=block), cuda(c.m0),
                                       cuda(dobs))
    finally:
        tpx.set_option(tpx.OPT_MATRIX_CORES, old)
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("ndim", [2, 3])
def test_fourth_order_stencil_paths(ndim):
    # space order 4 (R = 2): traces, the adjoint, and probed gradients on both
    # probing sides and on both contraction paths
    _print_case("order4", ndim=ndim)
    c = Case(small_2d(nz=40, nx=130, nt=200, nshots=3, nrec=13, order=4) if ndim == 2 else
             small_3d(nz=30, ny=13, nx=70, nt=80, nshots=2, nrec=8, order=4))
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, d_o) <= TOL
    rng = np.random.default_rng(8)
    d_in = rng.normal(size=d_o.shape).astype(np.float32).astype(np.float64)
    q_o = oracle.adjoint(c.ogrid(), c.m_true, c.src, c.rec, d_in)
    q_g = to_np(tpx.adjoint(c.tgrid(), c.tgeom(), cuda(c.m_true), cuda(d_in)))
    assert rel_l2(q_g, q_o) <= TOL
    dobs = d_o.astype(np.float32).astype(np.float64)
    for side, mfma in ((0, 1), (1, 2)):
        g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=32, seed=13, side=side)
        old = tpx.get_option(tpx.OPT_MATRIX_CORES)
        try:
            tpx.set_option(tpx.OPT_MATRIX_CORES, mfma)
            g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=32, seed=13, block=29, dtt_side=side),
                                           cuda(c.m0), cuda(dobs))
        finally:
            tpx.set_option(tpx.OPT_MATRIX_CORES, old)
        assert rel_l2(to_np(g_g), g_o) <= TOL
        assert abs(float(J_g.item()) - J_o) <= TOL * J_o
    # repeat calls are bitwise identical (the staged halo planes are not raced)
    probe = tpx.Probe(r=8, seed=2, block=17)
    runs = [to_np(tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))[0]) for _ in range(3)]
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], runs[2])


def _check_all_paths(c, r=16, seed=31):
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, d_o) <= TOL
    dobs = d_o.astype(np.float32).astype(np.float64)
    g_o, J_o = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_g, J_g = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=seed)
    for mfma in (1, 2):
        old = tpx.get_option(tpx.OPT_MATRIX_CORES)
        try:
            tpx.set_option(tpx.OPT_MATRIX_CORES, mfma)
            g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=r, seed=seed, block=23), cuda(c.m0),
                                           cuda(dobs))
        finally:
            tpx.set_option(tpx.OPT_MATRIX_CORES, old)
        assert rel_l2(to_np(g_g), g_o) <= TOL
        assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("ndim", [2, 3])
def test_no_absorbing_layer(ndim):
    # nbl = 0: the padded box is the physical grid, zero outside, no damping
    _print_case("nbl0", ndim=ndim)
    _check_all_paths(Case(small_2d(nz=30, nx=70, nt=150, nbl=0, nshots=2, nrec=9) if ndim == 2 else
                          small_3d(nz=20, ny=12, nx=30, nt=60, nbl=0, nshots=2, nrec=6)))


@pytest.mark.parametrize("ndim", [2, 3])
def test_grids_smaller_than_one_tile(ndim):
    _print_case("tiny", ndim=ndim)
    _check_all_paths(Case(small_2d(nz=6, nx=7, nt=60, nbl=2, nshots=2, nrec=3) if ndim == 2 else
                          small_3d(nz=5, ny=4, nx=6, nt=40, nbl=2, nshots=2, nrec=3)))


def test_24_shots_in_one_batch():
    # 24 shots: three shots per XCD group share each tile's beta
    _print_case("shots24")
    _check_all_paths(Case(small_2d(nz=30, nx=60, nt=120, nshots=24, nrec=7)))


def test_identity_and_orthonormal_probes_give_exact_gradient():
    c = Case(small_2d(nz=30, nx=70, nt=120, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    g_o, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_id, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(kind="identity", r=c.wl.nt), cuda(c.m0),
                                  cuda(dobs))
    assert rel_l2(to_np(g_id), g_o) <= TOL
    from scipy.fft import dct
    Q = dct(np.eye(c.wl.nt), norm="ortho", axis=0)
    Zs = np.stack([Q] * c.wl.nshots)
    g_q, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(),
                                 tpx.Probe(kind="explicit", r=c.wl.nt, Z=cuda(Zs), scale=1.0), cuda(c.m0),
                                 cuda(dobs))
    assert rel_l2(to_np(g_q), g_o) <= 2 * TOL


def test_split_forward_backward_equals_gradient_call():
    c = Case(small_2d(nz=30, nx=80, nt=140, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    probe = tpx.Probe(r=8, seed=3)
    g1, J1, d1 = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs), return_traces=True)
    d, state = tpx.forward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0))
    assert np.array_equal(to_np(d), to_np(d1))
    g2 = tpx.backward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), d - cuda(dobs), state)
    assert np.array_equal(to_np(g1), to_np(g2))


def test_backward_reports_a_state_from_another_probe_set():
    # the state carries the identity of the forward pass that wrote it; the
    # backward pass compares it on the device and tpx_check_workspace reports
    # a mismatch (other seed, other r with the same state size, other side)
    import torch
    c = Case(small_2d(nz=30, nx=60, nt=100, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    m, d = cuda(c.m0), cuda(dobs)
    p5 = tpx.Probe(r=8, seed=5)
    dsp, state = tpx.forward_probed(c.tgrid(), c.tgeom(), p5, m)
    ws = tpx.alloc_workspace(tpx.CALL_BACKWARD_PROBED, c.tgrid(), c.tgeom(), p5)
    tpx.backward_probed(c.tgrid(), c.tgeom(), p5, m, dsp - d, state, ws=ws)
    tpx.check_workspace(ws)
    for other in (tpx.Probe(r=8, seed=6), tpx.Probe(r=8, seed=5, dtt_side=1), tpx.Probe(r=8, seed=5, kind="gauss_b64")):
        ws2 = tpx.alloc_workspace(tpx.CALL_BACKWARD_PROBED, c.tgrid(), c.tgeom(), other)
        tpx.backward_probed(c.tgrid(), c.tgeom(), other, m, dsp - d, state, ws=ws2)
        with pytest.raises(tpx.TpxError) as e:
            tpx.check_workspace(ws2)
        assert e.value.status == tpx.E_STATE
    torch.cuda.synchronize()


def test_concurrent_host_threads():
    # four host threads, each with its own stream, problem and workspace, call
    # the library at once (ctypes releases the GIL); every result equals the
    # single-threaded one bit for bit
    import threading
    import torch
    _print_case("threads")
    cases = [Case(small_2d(nz=30, nx=60 + 10 * i, nt=120, nshots=2, nrec=7, seed=40 + i)) for i in range(2)] + \
            [Case(small_3d(nz=16, ny=10, nx=24 + 6 * i, nt=50, nshots=1, nrec=5, seed=50 + i)) for i in range(2)]
    inputs = [(c, cuda(c.m0), cuda(c.dobs_oracle()), tpx.Probe(r=16 * (1 + i % 2), seed=i, block=17))
              for i, c in enumerate(cases)]
    ref = [tpx.gradient_probed(c.tgrid(), c.tgeom(), p, m, d) for c, m, d, p in inputs]
    torch.cuda.synchronize()
    out = [None] * len(inputs)
    errors = []

    def work(i):
        try:
            c, m, d, p = inputs[i]
            s = torch.cuda.Stream()
            res = []
            for _ in range(3):
                with torch.cuda.stream(s):
                    res.append(tpx.gradient_probed(c.tgrid(), c.tgeom(), p, m, d, stream=s))
            s.synchronize()
            out[i] = res
        except Exception as e:   # reported below, on the test's thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(inputs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i, res in enumerate(out):
        for g, J in res:
            assert torch.equal(g, ref[i][0]) and torch.equal(J, ref[i][1]), i


@pytest.mark.parametrize("ndim", [2, 3])
def test_deterministic_bitwise(ndim):
    # every kernel family twice on fresh workspaces (stale contents differ):
    # identical bits catch races in LDS staging and uninitialised reads
    import torch
    _print_case("determinism", ndim=ndim)
    c = _grad_case(ndim)
    dobs = c.dobs_oracle()
    m, d = cuda(c.m0), cuda(dobs)
    calls = [
        lambda: tpx.forward(c.tgrid(), c.tgeom(), m),
        lambda: tpx.adjoint(c.tgrid(), c.tgeom(), m, d),
        lambda: tpx.gradient_full(c.tgrid(), c.tgeom(), m, d),
        lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=8, seed=9), m, d),
        lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=64, seed=9, block=33), m, d),
        lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(),
                                    tpx.Probe(r=16, seed=9, keep_vbar=True, imaging=1, dtt_side=1), m, d),
        lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(kind="range_finder", r=4, seed=9), m, d),
    ]
    for i, call in enumerate(calls):
        first = call()
        torch.cuda.synchronize()
        junk = torch.full((1 << 26,), float("nan"), device="cuda")   # dirty the allocator's cached blocks
        del junk
        second = call()
        first = first if isinstance(first, tuple) else (first,)
        second = second if isinstance(second, tuple) else (second,)
        for x, y in zip(first, second):
            assert torch.equal(x, y), i


def test_workspace_flags_bad_model():
    c = Case(small_2d(nz=20, nx=20, nt=20, nshots=1, nrec=3))
    m = c.m_true.copy()
    m[3, 4] = -1.0
    ws = tpx.alloc_workspace(tpx.CALL_FORWARD, c.tgrid(), c.tgeom())
    tpx.forward(c.tgrid(), c.tgeom(), cuda(m), ws=ws)
    with pytest.raises(tpx.TpxError) as e:
        tpx.check_workspace(ws)
    assert e.value.status == tpx.E_NUMERIC
    m = c.m_true.copy()
    m[3, 4] = 0.5 / c.wl.vmax ** 2   # velocity above damp_vmax
    tpx.forward(c.tgrid(), c.tgeom(), cuda(m), ws=ws)
    with pytest.raises(tpx.TpxError) as e:
        tpx.check_workspace(ws)
    assert e.value.status == tpx.E_CFL


# --------------------------------------------------------------------------- #
# measured configurations
# --------------------------------------------------------------------------- #

def test_c0_two_layer_full_and_probed():
    # 101 x 101, order 4, 1 shot, nt = 501, r = 8 Rademacher (seed 1)
    _print_case("c0")
    c = Case(workload("c0_two_layer_2d"))
    dobs = c.dobs_oracle()
    g_o, J_o = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_g, J_g = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    gp_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=c.wl.probe_seed)
    gp_g, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=8, seed=c.wl.probe_seed), cuda(c.m0),
                                  cuda(dobs))
    assert rel_l2(to_np(gp_g), gp_o) <= TOL


def test_3d_sources_across_z_chunk_boundary_and_dense_receivers():
    # receivers straddle the boundary between the second and third 12-plane z
    # chunks (padded z = 23.5) and sit 0.37 h apart, so several share injection nodes
    wl = small_3d(nz=48, ny=12, nx=40, nt=80, nbl=5, nshots=2, nrec=4)
    zc = (24 - wl.nbl - 0.5) * wl.h
    rec = [(3.0 + 0.37 * wl.h * i, 0.5 * (wl.shape[1] - 1) * wl.h, zc) for i in range(30)]
    wl = wl.with_(rec=rec)
    _print_case("3d_chunk_boundary")
    c = Case(wl)
    dobs = c.dobs_oracle()
    d_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    assert rel_l2(d_g, dobs) <= TOL
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=2)
    g_g, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=8, seed=2, block=7), cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL


def test_2d_dense_off_grid_receivers():
    wl = small_2d(nz=30, nx=90, nt=150, nshots=2, nrec=4)
    rec = [(5.0 + 0.37 * wl.h * i, 0.0, 3.3 * wl.h) for i in range(150)]
    wl = wl.with_(rec=rec)
    c = Case(wl)
    dobs = c.dobs_oracle()
    g_o, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_g, _ = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL


# the FP64 oracle of the full configuration takes minutes of CPU time
@pytest.mark.timeout(300)
def test_c1_full_configuration():
    # 801 x 301, 16 shots batched in one launch, order 8, nt = 2401, r = 16
    # Rademacher (the benchmarked launch configuration), against the oracle
    _print_case("c1_full")
    wl = workload("c1_layered_2d_16shots")
    c = Case(wl)
    # the observed data come from the oracle; the library's traces of the
    # true model must match them shot by shot
    dobs = c.dobs_oracle()
    d_true_g = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    for s in range(wl.nshots):
        assert rel_l2(d_true_g[s], dobs[s]) <= TOL, s
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=wl.r, seed=wl.probe_seed)
    g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=wl.r, seed=wl.probe_seed), cuda(c.m0),
                                   cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


# source positions (x, y, z in metres) on the 401 x 401 x 301 grid at 12.5 m:
# near the top face; at mid depth next to the x = max and y = 0 faces; at the
# bottom next to the x = 0, y = max and z = max faces.  Each one's 40-step
# record reaches the absorbing layer of its faces and spans two or three z
# chunks of both step kernels, so the three together cover all six faces and
# the first, middle and last chunks.
C3_SOURCES = [(2500.0, 2500.0, 50.0), (4930.0, 70.0, 1880.0), (60.0, 4940.0, 3690.0)]


@pytest.mark.parametrize("src", C3_SOURCES)
def test_c3_full_grid_truncated_record(src):
    # 401 x 401 x 301 at 12.5 m (the 3D configuration's grid and launch shape),
    # r = 32; record truncated to 40 steps (30 Hz wavelet) so the FP64 oracle
    # finishes in about a minute; receivers around the source; the gradient is
    # compared at 4096 points around the source computed by the oracle one by
    # one, for one-step and for fused two-step 3D launches.
    import torch
    _print_case("c3_truncated", src=src)
    wl = workload("c3_layered_3d").with_(nt=40, f_khz=0.03)
    h = wl.h
    nz, ny, nx = wl.shape
    ext = [(nx - 1) * h, (ny - 1) * h, (nz - 1) * h]
    rec = [tuple(min(max(src[a] + off[a], 0.0), ext[a]) for a in range(3))
           for off in [(dx * 2.3 * h, dy * 2.1 * h, dz * 1.9 * h) for dx in (-2, 0, 2) for dy in (-2, 0, 2)
                       for dz in (-1, 1)]]
    wl = wl.with_(src=[src], rec=rec)
    c = Case(wl)
    d_o = oracle.forward(c.ogrid(), c.m_true, c.src, c.rec, c.wav)
    dobs = np.zeros_like(d_o)
    rng = np.random.default_rng(0)
    ci = [int(round(src[a] / h)) for a in range(3)]   # x, y, z indices of the source
    lo = [max(ci[a] - 12, 0) for a in range(3)]
    hi = [min(ci[a] + 13, (nx, ny, nz)[a]) for a in range(3)]
    xx, yy, zz = (rng.integers(lo[a], hi[a], 4096) for a in range(3))
    pts = (zz * ny + yy) * nx + xx
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=wl.r, seed=wl.probe_seed,
                                      points=pts)
    assert np.linalg.norm(g_o) > 0
    print("[c3] points on faces (x, y, z):",
          [int(np.sum(v == 0)) + int(np.sum(v == n - 1)) for v, n in ((xx, nx), (yy, ny), (zz, nz))], flush=True)
    for fused in (0, 1):
        try:
            tpx.set_option(tpx.OPT_FUSED_STEPS_3D, fused)
            d_g = tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true))
            g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=wl.r, seed=wl.probe_seed), cuda(c.m0),
                                           cuda(dobs))
            torch.cuda.synchronize()
        finally:
            tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 0)
        g_s = g_g.reshape(-1).index_select(0, torch.as_tensor(pts, device="cuda")).double().cpu().numpy()
        del g_g
        print("[c3] fused", fused, "traces rel", rel_l2(to_np(d_g), d_o), "gradient rel", rel_l2(g_s, g_o),
              flush=True)
        assert rel_l2(to_np(d_g), d_o) <= TOL
        assert rel_l2(g_s, g_o) <= TOL
        assert abs(float(J_g.item()) - J_o) <= TOL * J_o


def test_c3_full_grid_dot_test_and_whole_gradient():
    # Properties that hold at any size, on the full 401 x 401 x 301 grid over
    # every tile, z chunk and damped face of both 3D step kernels: four shots at
    # depths in the first, middle and last chunks, receivers on a lattice every
    # 24 nodes through the whole volume, faces included (4536 of them), a
    # 60-step record.
    # - adjoint dot test <F q, d> = <q, F^T d> with random q and d;
    # - the whole probed gradient and all traces, one-step against two-step
    #   launches, bit for bit.
    import torch
    _print_case("c3_dot_whole")
    wl = workload("c3_layered_3d").with_(nt=60)
    h = wl.h
    nz, ny, nx = wl.shape
    src = [(2500.0, 2500.0, 60.0), (4987.5, 12.5, 1875.0), (30.0, 4970.0, 3740.0), (1250.0, 3750.0, 2500.0)]
    lat = lambda n: [i * h for i in range(0, n, 24)] + ([(n - 1) * h] if (n - 1) % 24 else [])
    rec = [(x, y, z) for z in lat(nz) for y in lat(ny) for x in lat(nx)]
    wl = wl.with_(src=src, rec=rec)
    c = Case(wl)
    rng = np.random.default_rng(12)
    S, nt, nrec = wl.nshots, wl.nt, len(rec)
    q = rng.normal(size=(S, nt)).astype(np.float32)
    d_in = rng.normal(size=(S, nt, nrec)).astype(np.float32)
    geom_q = tpx.Geometry(c.src, c.rec, cuda(q))
    m = cuda(c.m_true)
    Fq = to_np(tpx.forward(c.tgrid(), geom_q, m))
    FTd = to_np(tpx.adjoint(c.tgrid(), geom_q, m, cuda(d_in)))
    lhs, rhs = float(np.sum(Fq * d_in.astype(np.float64))), float(np.sum(q.astype(np.float64) * FTd))
    print(f"[c3_dot] receivers {nrec}, <Fq,d> {lhs:.6e}, <q,F^T d> {rhs:.6e}", flush=True)
    assert abs(lhs) > 0 and abs(lhs - rhs) <= 1e-4 * abs(lhs)
    # whole gradient and traces: one-step against two-step launches
    dobs = cuda(np.zeros((S, nt, nrec), dtype=np.float32))
    out = []
    for fused in (0, 1):
        try:
            tpx.set_option(tpx.OPT_FUSED_STEPS_3D, fused)
            d_g = tpx.forward(c.tgrid(), c.tgeom(), m)
            g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=8, seed=3), cuda(c.m0), dobs)
            torch.cuda.synchronize()
        finally:
            tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 0)
        out.append((d_g, g_g, float(J_g.item())))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]
    nz_frac = float((out[0][1] != 0).float().mean().item())
    print(f"[c3_dot] gradient nonzero fraction {nz_frac:.3f}", flush=True)
    assert nz_frac > 0.01


def test_largest_2d_shot_fields():
    # Two shots of 5,200,000 x 100 nodes: each padded shot field holds 1.0e9
    # floats (93% of the 2^30 limit), so in-shot byte offsets pass 2^31 and the
    # second shot starts 4 GB into each ring slot.  Shot 0 sits in interior
    # (fast-path) tiles, shot 1 in the bottom absorbing layer's tiles; one
    # receiver lies on the last physical column, one on the bottom-left corner.
    # A slow block around each source scatters 30% of the traces within the
    # 8-step record, which keeps the FP64 oracle to about a minute.  The
    # gradient is compared on the 5,000 nodes around the sources, with the
    # contractions on the vector units (default at r = 16) and on the matrix
    # cores.
    import torch
    nz, nx, h, nt = 5_200_000, 100, 10.0, 8
    _print_case("largest_2d", nz=nz, nx=nx, nshots=2, nt=nt)
    xs, zs = [500.0, 300.0], [(nz - 200) * h, (nz - 30) * h]
    src = np.array([[x, 0.0, z] for x, z in zip(xs, zs)])
    rec = np.array([[[x + dx, 0.0, z + dz] for dx, dz in ((-33.0, 27.0), (41.0, -12.5), (0.0, 50.0),
                                                           (-47.5, -40.0), (12.5, 0.0))] +
                    [[990.0, 0.0, z + 5.0] if i == 0 else [0.0, 0.0, (nz - 1) * h]]
                    for i, (x, z) in enumerate(zip(xs, zs))])
    rng = np.random.default_rng(2)
    wav = rng.standard_normal((2, nt)).astype(np.float32).astype(np.float64)
    m_true = np.full((nz, nx), 0.25)
    for x, z in zip(xs, zs):
        r0, c0 = int(z / h), int(x / h)
        m_true[r0 - 6:r0 + 7, c0 - 10:c0 + 11] = 0.3125
    m0 = np.full((nz, nx), 0.25)
    og = oracle.Grid((nz, nx), h=h, dt=1.5, nt=nt, order=8, nbl=20, damp_vmax=3.0)
    tg = tpx.Grid((nz, nx), h=h, dt=1.5, nt=nt, order=8, nbl=20, damp_vmax=3.0)
    geom = tpx.Geometry(src, rec, cuda(wav))
    dobs = oracle.forward(og, m_true, src, rec, wav).astype(np.float32).astype(np.float64)
    d_g = to_np(tpx.forward(tg, geom, cuda(m_true)))
    del m_true
    assert rel_l2(d_g, dobs) <= TOL
    pts = np.concatenate([np.arange((int(z / h) - 12) * nx, (int(z / h) + 13) * nx) for z in zs])
    g_o, J_o = oracle.gradient_probed(og, m0, src, rec, wav, dobs, r=16, seed=9, points=pts)
    assert np.linalg.norm(g_o) > 0 and J_o > 1e-3 * 0.5 * float(np.sum(dobs ** 2))
    probe = tpx.Probe(r=16, seed=9)
    m0_d, dobs_d = cuda(m0), cuda(dobs)
    del m0
    ws = tpx.alloc_workspace(tpx.CALL_GRADIENT_PROBED, tg, geom, probe)
    sel = torch.as_tensor(pts, device="cuda")
    for option in (1, 2):
        old = tpx.get_option(tpx.OPT_MATRIX_CORES)
        try:
            tpx.set_option(tpx.OPT_MATRIX_CORES, option)
            g_g, J_g = tpx.gradient_probed(tg, geom, probe, m0_d, dobs_d, ws=ws)
        finally:
            tpx.set_option(tpx.OPT_MATRIX_CORES, old)
        g_s = g_g.reshape(-1).index_select(0, sel).double().cpu().numpy()
        del g_g
        print("[largest_2d] option", option, "rel", rel_l2(g_s, g_o), flush=True)
        assert rel_l2(g_s, g_o) <= TOL
        assert abs(float(J_g.item()) - J_o) <= TOL * J_o


def test_largest_3d_shot_field():
    # One shot of 100,000 x 30 x 30 nodes: the padded field holds 1.0e9 floats
    # (128 x 78 x 100,048, 93% of the 2^30 limit), so plane offsets pass 2^31
    # bytes; the source sits 100 planes above the bottom, inside a slow block.
    import torch
    nz, ny, nx, h, nt = 100_000, 30, 30, 10.0, 8
    _print_case("largest_3d", nz=nz, ny=ny, nx=nx, nt=nt)
    x, y, z = 150.0, 145.0, (nz - 100) * h
    src = np.array([[x, y, z]])
    rec = np.array([[[x + dx, y + dy, z + dz] for dx, dy, dz in ((-33.0, 12.5, 27.0), (41.0, 0.0, -12.5),
                                                                  (0.0, -20.0, 45.0), (12.5, 7.5, 0.0))] +
                    [[290.0, 290.0, (nz - 1) * h]]])
    rng = np.random.default_rng(3)
    wav = rng.standard_normal((1, nt)).astype(np.float32).astype(np.float64)
    m_true = np.full((nz, ny, nx), 0.25)
    r0, c0, y0 = int(z / h), int(x / h), int(y / h)
    m_true[r0 - 5:r0 + 6, y0 - 5:y0 + 6, c0 - 5:c0 + 6] = 0.3125
    m0 = np.full((nz, ny, nx), 0.25)
    og = oracle.Grid((nz, ny, nx), h=h, dt=1.0, nt=nt, order=8, nbl=20, damp_vmax=3.0)
    tg = tpx.Grid((nz, ny, nx), h=h, dt=1.0, nt=nt, order=8, nbl=20, damp_vmax=3.0)
    geom = tpx.Geometry(src, rec, cuda(wav))
    dobs = oracle.forward(og, m_true, src, rec, wav).astype(np.float32).astype(np.float64)
    d_g = to_np(tpx.forward(tg, geom, cuda(m_true)))
    del m_true
    assert rel_l2(d_g, dobs) <= TOL
    pts = np.arange((r0 - 8) * ny * nx, (r0 + 9) * ny * nx)
    g_o, J_o = oracle.gradient_probed(og, m0, src, rec, wav, dobs, r=16, seed=11, points=pts)
    assert np.linalg.norm(g_o) > 0 and J_o > 1e-3 * 0.5 * float(np.sum(dobs ** 2))
    g_g, J_g = tpx.gradient_probed(tg, geom, tpx.Probe(r=16, seed=11), cuda(m0), cuda(dobs))
    g_s = g_g.reshape(-1).index_select(0, torch.as_tensor(pts, device="cuda")).double().cpu().numpy()
    print("[largest_3d] rel", rel_l2(g_s, g_o), flush=True)
    assert rel_l2(g_s, g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("block", [16, 15])
def test_overlapped_contractions_are_bitwise_identical(block):
    # contractions on the auxiliary stream (ring of 2b + 3 slots) give the same
    # bits as in stream order: same kernels, same summation order, with fused
    # two-step launches paired differently around odd block ends
    _print_case("overlap_2d", block=block)
    c = Case(small_2d(nz=30, nx=90, nt=170, nshots=2, nrec=11))
    dobs = c.dobs_oracle()
    probe = tpx.Probe(r=8, seed=4, block=block)
    try:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 0)
        a, Ja = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
        full0, _ = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs))
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 1)
        b, Jb = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
        full1, _ = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs))
        job = tpx.Job(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
        while not job.advance(5):
            pass
        import torch
        torch.cuda.synchronize()
    finally:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 0)
    assert np.array_equal(to_np(a), to_np(b)) and float(Ja.item()) == float(Jb.item())
    assert np.array_equal(to_np(full0), to_np(full1))
    assert np.array_equal(to_np(job.g), to_np(a))


def test_3d_split_job_and_overlap_are_bitwise_identical():
    # 3D: the split forward/backward pair, a job advanced in chunks, and the
    # contractions overlapped on the auxiliary stream reproduce the gradient
    # call bit for bit (matrix-core fold at r = 32, ragged 19-level blocks)
    import torch
    _print_case("split_job_overlap_3d")
    c = Case(small_3d(nz=30, ny=12, nx=40, nt=70, nshots=2, nrec=7))
    dobs = c.dobs_oracle()
    m, d = cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=32, seed=6, block=19)
    g, J = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d)
    dsp, state = tpx.forward_probed(c.tgrid(), c.tgeom(), probe, m)
    g_split = tpx.backward_probed(c.tgrid(), c.tgeom(), probe, m, dsp - d, state)
    job = tpx.Job(c.tgrid(), c.tgeom(), probe, m, d)
    while not job.advance(9):
        pass
    try:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 1)
        g_ovl, J_ovl = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d)
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 1)
        g_ovl2, J_ovl2 = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d)
    finally:
        tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 0)
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 0)
    torch.cuda.synchronize()
    assert torch.equal(g_split, g) and torch.equal(job.g, g) and torch.equal(job.J, J)
    assert torch.equal(g_ovl, g) and torch.equal(J_ovl, J)
    assert torch.equal(g_ovl2, g) and torch.equal(J_ovl2, J)
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=32, seed=6)
    assert rel_l2(to_np(g), g_o) <= TOL


def test_all_tile_heights_agree():
    # 300 x 400 gives 80 tiles of 32 rows per shot: 8 shots (640) take 32-row
    # tiles, 5 shots (400) 16-row tiles and 4 shots (320) 8-row tiles.  Each
    # shot's traces are bitwise the same every way; the 8-shot gradient matches
    # the oracle.
    import torch
    _print_case("tile_heights")
    wl = small_2d(nz=300, nx=400, nt=160, nshots=8, nrec=21, seed=14)
    c8 = Case(wl)
    d8 = tpx.forward(c8.tgrid(), c8.tgeom(), cuda(c8.m_true))
    for n in (5, 4):
        cn = Case(wl, shots=range(n))
        dn = tpx.forward(cn.tgrid(), cn.tgeom(), cuda(c8.m_true))
        assert torch.equal(d8[:n], dn), n
    dobs = c8.dobs_oracle()
    assert rel_l2(to_np(d8), dobs) <= TOL
    g_o, J_o = oracle.gradient_probed(c8.ogrid(), c8.m0, c8.src, c8.rec, c8.wav, dobs, r=16, seed=3)
    g_g, J_g = tpx.gradient_probed(c8.tgrid(), c8.tgeom(), tpx.Probe(r=16, seed=3, block=41), cuda(c8.m0),
                                   cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


def test_one_and_two_step_launches_are_bitwise_identical():
    import torch

    # A job advanced one time step per call runs only one-step launches; the
    # gradient call fuses steps in pairs (odd nt leaves a single step at the
    # end of each pass).  Rounding is pinned, so both give the same bits.
    print("[case] one-step vs two-step launches, 2D", flush=True)
    c = Case(small_2d(nz=45, nx=130, nt=151, nshots=3, nrec=17))
    dobs = c.dobs_oracle()
    probe = tpx.Probe(r=8, seed=5, block=16)
    g2, J2 = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    job = tpx.Job(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    while not job.advance(1):
        pass
    torch.cuda.synchronize()
    assert torch.equal(job.g, g2) and torch.equal(job.J, J2)
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=5)
    assert rel_l2(to_np(g2), g_o) <= 1e-4


@pytest.mark.parametrize("order", [8, 4])
def test_3d_one_and_two_step_launches_are_bitwise_identical(order):
    import torch

    # 3D: a job advanced one time step per call runs only the one-step kernel;
    # with fused 3D steps switched on, the gradient call and the plain forward
    # run the two-step kernel (tiles of 16 rows, z chunks of 9 planes here,
    # interior blocks on the fast path, an odd record leaving one single step
    # per pass).  Same bits both ways, and the same as with the option off.
    print("[case] one-step vs two-step launches, 3D, order", order, flush=True)
    wl = small_3d(nz=60, ny=40, nx=130, nt=81, nbl=5, nshots=2, nrec=23, order=order)
    # receivers straddling x and y tile edges (x = 56, y = 16 padded nodes)
    rec = [(h * (56 - 5 - 1.5 + 0.7 * i), h * (16 - 5 - 0.5 + 0.45 * i), 0.12 * 59 * h) for i in range(8)
           for h in (wl.h,)]
    wl = wl.with_(rec=rec + [tuple(r) for r in wl.rec[:15]])
    c = Case(wl)
    dobs = c.dobs_oracle()
    m0, d = cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=8, seed=5, block=16)
    try:
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 1)
        d_two = tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true))
        g2, J2 = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m0, d)
        gf2, Jf2 = tpx.gradient_full(c.tgrid(), c.tgeom(), m0, d)
        job = tpx.Job(c.tgrid(), c.tgeom(), probe, m0, d)
        while not job.advance(1):
            pass
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 0)
        d_one = tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true))
        g1, J1 = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m0, d)
        torch.cuda.synchronize()
    finally:
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, 0)
    assert rel_l2(to_np(d_two), dobs) <= TOL
    assert torch.equal(d_one, d_two)
    assert torch.equal(job.g, g2) and torch.equal(job.J, J2)
    assert torch.equal(g1, g2) and torch.equal(J1, J2)
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=8, seed=5)
    assert rel_l2(to_np(g2), g_o) <= TOL
    assert abs(float(J2.item()) - J_o) <= TOL * J_o
    gf_o, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    assert rel_l2(to_np(gf2), gf_o) <= TOL


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("keep_vbar", [False, True])
def test_algorithm1_side_matches_oracle(ndim, keep_vbar):
    # dtt_side = 1: the forward pass probes the second time difference of u,
    # the adjoint pass probes lam itself (Algorithm 1 as printed)
    _print_case("grad_probed_dtt1", ndim=ndim, keep_vbar=keep_vbar)
    c = _grad_case(ndim)
    dobs = c.dobs_oracle()
    r, seed = 6, 91
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=seed, side=1)
    g_n, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=seed, side=0)
    assert rel_l2(g_n, g_o) > 1e-3   # the two sides are different estimators
    probe = tpx.Probe(r=r, seed=seed, block=13, keep_vbar=keep_vbar, dtt_side=1)  # ragged time blocks
    g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


def test_algorithm1_side_is_exact_with_identity_probes():
    _print_case("grad_identity_dtt1")
    c = Case(small_2d(nz=30, nx=70, nt=121, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    g_o, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    probe = tpx.Probe(kind="identity", r=c.wl.nt, dtt_side=1, block=16)
    g_id, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_id), g_o) <= TOL
    # the split autograd path carries the side through its saved state
    d, state = tpx.forward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0))
    res = d - cuda(dobs)
    g_split = tpx.backward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), res, state)
    assert rel_l2(to_np(g_split), to_np(g_id)) <= 1e-6


@pytest.mark.parametrize("ndim", [2, 3])
def test_range_finder_probes_match_oracle(ndim):
    # Q = qr(D D^T Z) per shot (Eq. 6): the GPU's FP64 Householder factor spans
    # the oracle's (NumPy) one; the probed gradient depends on Q Q^T only
    _print_case("range_finder", ndim=ndim)
    import torch
    c = _grad_case(ndim)
    dobs = c.dobs_oracle().astype(np.float32)
    # r within the numerical rank of D D^T Z: beyond it Q's columns are an
    # arbitrary orthonormal completion (the short 3D record reaches few
    # receivers: its traces have only ~4 significant singular values)
    r, seed = (6 if ndim == 2 else 3), 17
    Qo = oracle.range_finder_probes(dobs, r, seed)
    probe = tpx.Probe(kind="range_finder", r=r, seed=seed, block=13)
    Qg = to_np(tpx.range_finder_probes(c.tgrid(), c.tgeom(), probe, cuda(dobs))).astype(np.float64)
    for s in range(c.wl.nshots):
        assert np.abs(Qg[s].T @ Qg[s] - np.eye(r)).max() <= 1e-6
        assert np.linalg.norm(Qg[s] @ Qg[s].T - Qo[s] @ Qo[s].T) <= 1e-5 * np.sqrt(r)
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind="explicit", r=r, Z=Qo,
                                      scale=1.0)
    g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o
    # the split forward/backward pair with the same Q as explicit probes
    if ndim == 2:
        pe = tpx.Probe(kind="explicit", r=r, Z=cuda(Qg.astype(np.float32)), scale=1.0, block=13)
        d, state = tpx.forward_probed(c.tgrid(), c.tgeom(), pe, cuda(c.m0))
        g_split = tpx.backward_probed(c.tgrid(), c.tgeom(), pe, cuda(c.m0), d - cuda(dobs), state)
        assert torch.equal(g_split, g_g)


@pytest.mark.parametrize("r", [16, 64])
def test_range_finder_probes_at_large_r(r):
    # Eq. 6 with many probes: 70 receivers of random observed traces (full rank)
    # over 1200 samples, so Q is well determined; the tall-skinny QR runs over 9
    # panels (r = 16) or 4 (r = 64), and the gradient's contractions with Q run
    # on the matrix cores (split probes)
    _print_case("range_finder_large_r", r=r)
    import torch
    c = Case(small_2d(nz=30, nx=80, nt=1200, nshots=2, nrec=70))
    dobs = np.random.default_rng(r).standard_normal((2, 1200, 70)).astype(np.float32).astype(np.float64)
    Qo = oracle.range_finder_probes(dobs, r, 23)
    probe = tpx.Probe(kind="range_finder", r=r, seed=23)
    Qg = to_np(tpx.range_finder_probes(c.tgrid(), c.tgeom(), probe, cuda(dobs)))
    for s in range(2):
        assert np.abs(Qg[s].T @ Qg[s] - np.eye(r)).max() <= 1e-5
        assert np.linalg.norm(Qg[s] @ Qg[s].T - Qo[s] @ Qo[s].T) <= 1e-5 * np.sqrt(r)
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind="explicit", r=r, Z=Qo,
                                      scale=1.0)
    g_g, J_g = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o
    assert torch.isfinite(g_g).all()


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_imaging_condition_matches_oracle(ndim):
    # Eq. 5: the space-only operator grad applied to the r probed fields
    _print_case("imaging_graddot", ndim=ndim)
    c = _grad_case(ndim)
    dobs = c.dobs_oracle()
    r, seed = 6, 29
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=seed, imaging=1)
    probe = tpx.Probe(r=r, seed=seed, block=13, keep_vbar=True, imaging=1)
    g_g, _ = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    # the split pair images the same way
    d, state = tpx.forward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0))
    g_split = tpx.backward_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), d - cuda(dobs), state)
    assert rel_l2(to_np(g_split), g_o) <= TOL
