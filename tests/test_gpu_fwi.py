"""GPU tests of the inversion loop (Example section): the objective call
against the oracle, and SPG iterations driven by the library's probed gradient
against the same iterations driven by the FP64 oracle (oracle/spg.py) on
identical seeded inputs and shot batches."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-4

if gpu_available():
    ensure_built()

import oracle  # noqa: E402
from oracle import spg as ospg  # noqa: E402
from paper_2104_00794_amd import fwi, tpx  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d  # noqa: E402


def _print_case(name, **kw):
    print("[case]", name, kw, flush=True)


def _oracle_J(c, m, idx, dobs):
    d = oracle.forward(c.ogrid(), m, c.src[idx], c.rec[idx], c.wav[idx])
    return 0.5 * float(np.sum((d - dobs[idx]) ** 2))


def test_objective_matches_oracle_and_the_gradient_call():
    _print_case("objective", nz=40, nx=90, nshots=3)
    c = Case(small_2d(nz=40, nx=90, nt=200, nshots=3, nrec=11, order=8))
    dobs = c.dobs_oracle()
    idx = np.arange(3)
    J_o = _oracle_J(c, c.m0, idx, dobs)
    m, d_obs = cuda(c.m0), cuda(dobs)
    J, d = tpx.objective(c.tgrid(), c.tgeom(), m, d_obs, return_traces=True)
    assert abs(float(J.item()) - J_o) <= TOL * J_o
    # the same forward kernels and residual reduction as the gradient call: bitwise
    _, J2, d2 = tpx.gradient_probed(c.tgrid(), c.tgeom(), tpx.Probe(r=8, seed=4), m, d_obs, return_traces=True)
    assert float(J.item()) == float(J2.item())
    assert np.array_equal(to_np(d), to_np(d2))
    assert np.array_equal(to_np(d), to_np(tpx.forward(c.tgrid(), c.tgeom(), m)))


@pytest.mark.parametrize("gradient", ["rademacher:8", "exact"])
def test_spg_iterations_match_the_oracle(gradient):
    kind, r = fwi.parse_gradient(gradient)
    _print_case("spg", gradient=gradient, nz=40, nx=64, nshots=4, batch=2, iters=3)
    c = Case(small_2d(nz=40, nx=64, nt=180, nshots=4, nrec=12, order=8, seed=9))
    dobs = c.dobs_oracle()
    lo, hi = 1.0 / c.wl.vmax ** 2, 1.0 / c.wl.vmin ** 2
    plan = fwi.batches(4, 2, 3, seed=1)
    seed0 = 40
    opts = fwi.SPGOptions(iters=3)
    import torch
    d_dev = cuda(dobs)
    wav_dev = cuda(c.wav)

    def geom(idx):
        sel = torch.as_tensor(idx, dtype=torch.long, device="cuda")
        return tpx.Geometry(c.src[idx], c.rec[idx], wav_dev.index_select(0, sel).contiguous())

    def data(idx):
        return d_dev.index_select(0, torch.as_tensor(idx, dtype=torch.long, device="cuda")).contiguous()

    def fg_gpu(x, k):
        idx = plan[k]
        if kind == "exact":
            g, J = tpx.gradient_full(c.tgrid(), geom(idx), x, data(idx))
        else:
            g, J = tpx.gradient_probed(c.tgrid(), geom(idx), tpx.Probe(kind=kind, r=r, seed=seed0 + k), x, data(idx))
        return float(J.item()), g

    def f_gpu(x, k):
        return float(tpx.objective(c.tgrid(), geom(plan[k]), x, data(plan[k])).item())

    def fg_orc(x, k):
        idx = plan[k]
        if kind == "exact":
            g, J = oracle.gradient_full(c.ogrid(), x, c.src[idx], c.rec[idx], c.wav[idx], dobs[idx])
        else:
            g, J = oracle.gradient_probed(c.ogrid(), x, c.src[idx], c.rec[idx], c.wav[idx], dobs[idx], kind=kind,
                                          r=r, seed=seed0 + k)
        return J, g

    def f_orc(x, k):
        return _oracle_J(c, x, plan[k], dobs)

    res_g = fwi.spg(fg_gpu, f_gpu, cuda(c.m0), lo, hi, opts)
    res_o = ospg.spg(fg_orc, f_orc, c.m0, lo, hi, ospg.Options(iters=3))
    for hg, ho in zip(res_g.history, res_o.history):
        print("[iter] gpu", hg.f, hg.alpha, hg.t, hg.trials, "oracle", ho.f, ho.alpha, ho.t, ho.trials, flush=True)
        assert hg.trials == ho.trials
        assert abs(hg.f - ho.f) <= TOL * abs(ho.f)
        assert abs(hg.f_new - ho.f_new) <= TOL * abs(ho.f_new)
        assert abs(hg.alpha - ho.alpha) <= 10 * TOL * ho.alpha
    assert res_o.history[-1].f_new < res_o.history[0].f
    upd_o = res_o.x - c.m0
    assert np.linalg.norm(upd_o) > 1e-3 * np.linalg.norm(c.m0)      # the model moved
    assert rel_l2(to_np(res_g.x) - c.m0, upd_o) <= 10 * TOL


def test_probed_inversion_reduces_the_model_error():
    _print_case("invert", nz=60, nx=120, nshots=8, batch=4, iters=6)
    wl = small_2d(nz=60, nx=120, nt=400, nshots=8, nrec=40, order=8, seed=12)
    prob = fwi.Problem(wl)
    for spec in ("rademacher:16", "exact"):
        res, cnt = fwi.invert(prob, spec, fwi.SPGOptions(iters=6), batch=4, batch_seed=3, probe_seed=77)
        errs = [h.model_error for h in res.history]
        print("[invert]", spec, [round(e, 4) for e in errs], cnt, flush=True)
        assert errs[-1] < 0.98
        assert all(h.t > 0.0 for h in res.history)
        # the box, as its bounds round to the model's float32
        assert float(res.x.min()) >= float(np.float32(prob.lo)) and float(res.x.max()) <= float(np.float32(prob.hi))


def test_objective_edge_cases():
    import torch
    _print_case("objective_edges")
    c = Case(small_2d(nz=30, nx=40, nt=60, nshots=2, nrec=5, order=4))
    m = cuda(c.m0)
    # no receivers: nothing to misfit
    geom0 = tpx.Geometry(c.src, np.zeros((2, 0, 3)), cuda(c.wav))
    J0 = tpx.objective(c.tgrid(), geom0, m, torch.zeros((2, c.wl.nt, 0), device="cuda"))
    assert float(J0.item()) == 0.0
    # the observed data equal to the model's own traces: zero misfit, bitwise
    d = tpx.forward(c.tgrid(), c.tgeom(), m)
    assert float(tpx.objective(c.tgrid(), c.tgeom(), m, d).item()) == 0.0
    # the shortest record, two time levels
    c2 = Case(small_2d(nz=30, nx=40, nt=2, nshots=1, nrec=3, order=8))
    dob = np.ones((1, 2, 3))
    J2 = tpx.objective(c2.tgrid(), c2.tgeom(), cuda(c2.m0), cuda(dob))
    J2o = _oracle_J(c2, c2.m0, np.arange(1), dob)
    assert abs(float(J2.item()) - J2o) <= TOL * J2o
