"""Differentiation through the probed modelling operator (torch.autograd).

Workload: 401 x 201 at 10 m, 4 shots, order 8, nt = 2001, r = 32 Rademacher;
d_obs from the seeded true model, m0 its Gaussian-smoothed version.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built, rel_l2, to_np

pytestmark = pytest.mark.gpu

if gpu_available():
    ensure_built()

import torch  # noqa: E402

import oracle  # noqa: E402
from paper_2104_00794_amd import tpx  # noqa: E402
from paper_2104_00794_amd.autograd import exact_probe, misfit, modeling  # noqa: E402
from paper_2104_00794_amd.inputs import workload  # noqa: E402


def _edge_free(a):
    b = np.array(a, copy=True)
    b[0, :] = b[-1, :] = 0
    b[:, 0] = b[:, -1] = 0
    return b


def _loss_and_grad(c, m_np, probe):
    m = cuda(m_np).requires_grad_(True)
    d = modeling(m, c.tgrid(), c.tgeom(), probe)
    loss = misfit(d, cuda(c.dobs))
    loss.backward()
    return float(loss.item()), m.grad


@pytest.fixture(scope="module")
def c2():
    wl = workload("c2_autograd_2d")
    c = Case(wl)
    c.dobs = c.dobs_oracle()   # observed data from the oracle, fed to both sides
    return c


def test_backward_equals_probed_gradient_call(c2):
    print("[case] c2 autograd vs gradient call", flush=True)
    probe = tpx.Probe(r=32, seed=c2.wl.probe_seed)
    loss, grad = _loss_and_grad(c2, c2.m0, probe)
    g, J = tpx.gradient_probed(c2.tgrid(), c2.tgeom(), probe, cuda(c2.m0), cuda(c2.dobs))
    assert torch.equal(grad, g)
    assert loss == pytest.approx(float(J.item()), rel=1e-5)


def test_backward_matches_oracle(c2):
    print("[case] c2 autograd vs oracle", flush=True)
    probe = tpx.Probe(r=32, seed=c2.wl.probe_seed)
    _, grad = _loss_and_grad(c2, c2.m0, probe)
    g_o, _ = oracle.gradient_probed(c2.ogrid(), c2.m0, c2.src, c2.rec, c2.wav, c2.dobs, r=32,
                                    seed=c2.wl.probe_seed)
    assert rel_l2(to_np(grad), g_o) <= 1e-4


def test_exact_mode_taylor_and_finite_differences():
    # identity probes make the backward exact; shortened record keeps the
    # r = nt state (4 x 700 x 80,601 floats) small
    print("[case] c2 exact-mode Taylor", flush=True)
    c = Case(workload("c2_autograd_2d").with_(nt=700))
    c.dobs = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m_true)))
    loss0, grad = _loss_and_grad(c, c.m0, exact_probe(c.tgrid()))
    g_full, J_full = tpx.gradient_full(c.tgrid(), c.tgeom(), cuda(c.m0), cuda(c.dobs))
    assert rel_l2(to_np(grad), to_np(g_full)) <= 1e-4
    dm = _edge_free(c.m_true - c.m0)
    gdm = float(np.sum(to_np(grad) * dm))

    def J(h):
        d = to_np(tpx.forward(c.tgrid(), c.tgeom(), cuda(c.m0 + h * dm)))
        return 0.5 * float(np.sum((d - c.dobs) ** 2))

    J0 = J(0.0)
    # the full sweep h = 0.1 ... 9.8e-5 (halving).  The traces are FP32, so
    # the second-order remainder, which quarters per halving, reaches the
    # rounding of J after a few halvings; the ratios are asserted before that
    # and the h where the remainder stops quartering is printed.  Measured on
    # the GPU: ratios 3.8-4.2 down to h = 3.1e-3, rounding reached at h = 1.6e-3
    # (remainder about 1e-6 J0); the first-order ratios stay at 2.0 down to
    # 9.8e-5.  (The FP64 oracle holds the ratio 4 down to 1e-4: test_oracle_gradient.)
    hs = [0.1 / 2 ** i for i in range(11)]
    Jh = [J(h) for h in hs]
    r1 = [abs(j - J0) for j in Jh]
    r2 = [abs(j - J0 - h * gdm) for j, h in zip(Jh, hs)]
    q1 = [r1[i] / r1[i + 1] for i in range(len(hs) - 1)]
    q2 = [r2[i] / r2[i + 1] for i in range(len(hs) - 1)]
    sat = next((hs[i + 1] for i in range(len(q2)) if not 3.0 < q2[i] < 5.0), None)
    print("Taylor h", ["%.2e" % h for h in hs], flush=True)
    print("first-order ratios", ["%.3f" % q for q in q1], flush=True)
    print("second-order remainders / J0", ["%.2e" % (r / J0) for r in r2], flush=True)
    print("second-order ratios", ["%.3f" % q for q in q2], "; FP32 rounding reached at h =", sat, flush=True)
    assert all(1.7 < q < 2.3 for q in q1)
    assert all(3.0 < q < 5.0 for q in q2[:2])
    assert sat is None or sat < 0.0125
    # central finite difference of J along dm
    h = 0.01
    fd = (J(h) - J(-h)) / (2 * h)
    assert abs(fd - gdm) <= 2e-3 * abs(gdm), (fd, gdm)


def test_probed_directional_derivative(c2):
    # the probed gradient is unbiased; with r = 32 its directional derivative
    # along the model update stays close to the exact one
    print("[case] c2 probed directional error", flush=True)
    g_ex, _ = tpx.gradient_full(c2.tgrid(), c2.tgeom(), cuda(c2.m0), cuda(c2.dobs))
    dm = _edge_free(c2.m_true - c2.m0)
    ex = float(np.sum(to_np(g_ex) * dm))
    errs = []
    for seed in range(4):
        _, grad = _loss_and_grad(c2, c2.m0, tpx.Probe(r=32, seed=100 + seed))
        errs.append(abs(float(np.sum(to_np(grad) * dm)) - ex) / abs(ex))
    print("directional relative errors", errs, flush=True)
    assert np.mean(errs) < 0.25
