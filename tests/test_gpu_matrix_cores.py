"""GPU parity of the probe contractions on the matrix cores (bfloat16 MFMA,
each FP32 field value split exactly into three bfloat16 parts, FP32
accumulation) against the FP64 oracle, and against the FP32 vector-unit
contractions on the same inputs.  Time blocks of 37 levels start off the
16-level k tiles; r = 48 and 80 exercise partial probe chunks."""
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


def _case(ndim):
    if ndim == 2:
        return Case(small_2d(nz=40, nx=150, nt=220, nshots=3, nrec=17))
    return Case(small_3d(nz=40, ny=11, nx=70, nt=90, nshots=2, nrec=9))


def _with_option(value, fn):
    old = tpx.get_option(tpx.OPT_MATRIX_CORES)
    try:
        tpx.set_option(tpx.OPT_MATRIX_CORES, value)
        return fn()
    finally:
        tpx.set_option(tpx.OPT_MATRIX_CORES, old)


@pytest.mark.parametrize("ndim,kind,keep_vbar,side", [
    (2, "rademacher", False, 0), (2, "rademacher", True, 0), (2, "rademacher", False, 1), (2, "rademacher", True, 1),
    (2, "gauss_b64", False, 0), (2, "gauss_b64", True, 1),
    (3, "rademacher", False, 0), (3, "gauss_b64", True, 1),
])
def test_matrix_core_gradient_matches_oracle(ndim, kind, keep_vbar, side):
    _print_case("mfma_grad", ndim=ndim, kind=kind, keep_vbar=keep_vbar, side=side)
    c = _case(ndim)
    dobs = c.dobs_oracle()
    r, seed = 32, 61
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind=kind, r=r, seed=seed,
                                      side=side)
    probe = tpx.Probe(kind=kind, r=r, seed=seed, block=37, keep_vbar=keep_vbar, dtt_side=side)
    g_g, J_g = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs)))
    assert rel_l2(to_np(g_g), g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


@pytest.mark.parametrize("r", [16, 48, 64, 80])
def test_matrix_core_and_vector_contractions_agree(r):
    _print_case("mfma_vs_valu", r=r)
    c = Case(small_2d(nz=30, nx=90, nt=150, nshots=2, nrec=11))
    dobs = c.dobs_oracle()
    m, d = cuda(c.m0), cuda(dobs)
    for keep_vbar in (False, True):
        probe = tpx.Probe(r=r, seed=5, block=37, keep_vbar=keep_vbar)
        g_v, J_v = _with_option(0, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
        g_m, J_m = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
        assert float(J_v.item()) == float(J_m.item())   # the forward traces do not depend on the contraction
        assert rel_l2(to_np(g_m), to_np(g_v)) <= 1e-5
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=5)
    assert rel_l2(to_np(g_m), g_o) <= TOL


def test_matrix_core_split_and_job_paths_are_bitwise_equal():
    _print_case("mfma_split_job")
    c = Case(small_2d(nz=30, nx=70, nt=130, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    m, d = cuda(c.m0), cuda(dobs)
    probe = tpx.Probe(r=32, seed=8, block=21)

    def run():
        import torch
        g, J, dd = tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d, return_traces=True)
        dsp, state = tpx.forward_probed(c.tgrid(), c.tgeom(), probe, m)
        g_split = tpx.backward_probed(c.tgrid(), c.tgeom(), probe, m, dsp - d, state)
        job = tpx.Job(c.tgrid(), c.tgeom(), probe, m, d)
        while not job.advance(7):
            pass
        torch.cuda.synchronize()
        return g, g_split, job.g

    g, g_split, g_job = _with_option(1, run)
    assert np.array_equal(to_np(g), to_np(g_job))
    # the split pair images the same residual (d - d_obs) with the same kernels
    assert np.array_equal(to_np(g_split), to_np(g))


@pytest.mark.parametrize("r,keep_vbar,side", [(32, False, 0), (32, True, 1), (48, False, 1), (16, True, 0)])
def test_split_probes_on_the_matrix_cores_match_oracle(r, keep_vbar, side):
    # explicit probes with arbitrary FP32 entries: each probe value is split in
    # three bfloat16 parts as well (six products per tile)
    _print_case("mfma_split_probes", r=r, keep_vbar=keep_vbar, side=side)
    c = Case(small_2d(nz=40, nx=150, nt=220, nshots=3, nrec=17))
    dobs = c.dobs_oracle()
    rng = np.random.default_rng(r + 7)
    Z = rng.standard_normal((c.wl.nshots, c.wl.nt, r)).astype(np.float32).astype(np.float64)
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind="explicit", r=r, Z=Z,
                                    scale=1.0 / r, side=side)
    probe = tpx.Probe(kind="explicit", r=r, Z=cuda(Z), scale=1.0 / r, block=37, keep_vbar=keep_vbar, dtt_side=side)
    m, d = cuda(c.m0), cuda(dobs)
    g_m, _ = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
    g_v, _ = _with_option(0, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
    assert rel_l2(to_np(g_m), g_o) <= TOL
    assert rel_l2(to_np(g_m), to_np(g_v)) <= 1e-5


# the FP64 oracle of the full configuration takes minutes of CPU time
@pytest.mark.timeout(300)
def test_c1_r64_full_configuration_on_the_matrix_cores():
    # 801 x 301, 16 shots batched in one launch, order 8, nt = 2401, r = 64
    # Rademacher under the default option: the accumulation and the fold run on
    # the matrix cores over 1024-level blocks (the benchmarked r = 64 launch
    # configuration).  The gradient is compared at 4096 sampled points that the
    # oracle computes one by one, and the objective in full.
    _print_case("c1_r64_full")
    wl = workload("c1_layered_2d_16shots")
    c = Case(wl)
    dobs = c.dobs_oracle()
    r = 64
    nz, nx = wl.shape
    pts = np.sort(np.random.default_rng(64).choice(nz * nx, 4096, replace=False))
    g_o, J_o = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=r, seed=wl.probe_seed,
                                      points=pts)
    probe = tpx.Probe(r=r, seed=wl.probe_seed)
    g_g, J_g = _with_option(1, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs)))
    g_s = to_np(g_g).reshape(-1)[pts]
    assert np.linalg.norm(g_o) > 0
    assert rel_l2(g_s, g_o) <= TOL
    assert abs(float(J_g.item()) - J_o) <= TOL * J_o


def test_identity_probes_and_gradient_imaging_on_the_matrix_cores():
    # identity probes with r = nt = 128 (eight 16-level tiles, exact in
    # bfloat16) give the exact gradient; Eq. 5's imaging of vbar accumulated on
    # the matrix cores matches the oracle in 2D and 3D
    _print_case("mfma_identity_imaging")
    c = Case(small_2d(nz=30, nx=70, nt=128, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    g_full, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    g_id, _ = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(kind="identity", r=128),
                                                         cuda(c.m0), cuda(dobs)))
    assert rel_l2(to_np(g_id), g_full) <= TOL
    for ndim in (2, 3):
        c = _case(ndim)
        dobs = c.dobs_oracle()
        g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, r=16, seed=3, imaging=1)
        probe = tpx.Probe(r=16, seed=3, block=37, keep_vbar=True, imaging=1)
        g_g, _ = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, cuda(c.m0), cuda(dobs)))
        assert rel_l2(to_np(g_g), g_o) <= TOL


def test_misaligned_explicit_probes_fall_back_to_the_vector_units():
    # the matrix-core fold reads explicit probes as 16-byte vectors: a Z that
    # starts 4 bytes into its allocation takes the vector-unit contractions
    import torch
    _print_case("mfma_misaligned_Z")
    c = Case(small_2d(nz=30, nx=70, nt=100, nshots=2, nrec=9))
    dobs = c.dobs_oracle()
    r = 32
    Z = np.random.default_rng(5).standard_normal((2, 100, r)).astype(np.float32).astype(np.float64)
    buf = torch.zeros(Z.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = cuda(Z).reshape(-1)
    Zmis = buf[1:].view(2, 100, r)
    assert Zmis.data_ptr() % 16 != 0
    g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind="explicit", r=r, Z=Z,
                                    scale=1.0 / r)
    m, d = cuda(c.m0), cuda(dobs)
    for Zt in (cuda(Z), Zmis):
        probe = tpx.Probe(kind="explicit", r=r, Z=Zt, scale=1.0 / r, block=37)
        g_m, _ = _with_option(2, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
        assert rel_l2(to_np(g_m), g_o) <= TOL
    g_v, _ = _with_option(0, lambda: tpx.gradient_probed(c.tgrid(), c.tgeom(), probe, m, d))
    assert torch.equal(g_m, g_v)   # the misaligned call ran the vector-unit kernels
