"""GPU: the probed gradient is an unbiased estimator of the exact one
(Randomized trace estimation; Eq. 4).  Over many probe seeds the GPU's probed
gradients scatter around the oracle's exact gradient with the closed-form
Hutchinson variance, computed from the oracle's forward and adjoint histories,
and their running mean converges to the exact gradient like 1/N."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, cuda, ensure_built, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="no GPU")]

import oracle  # noqa: E402
from paper_2104_00794_amd import tpx  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d  # noqa: E402


@pytest.mark.parametrize("kind,kappa", [("rademacher", 1.0), ("gauss_b64", 3.0 - 2.0 / 64.0)])
def test_gpu_probed_gradient_mean_converges_with_hutchinson_variance(kind, kappa):
    ensure_built()
    print(f"[probe_statistics] kind={kind}", flush=True)
    c = Case(small_2d(nz=16, nx=18, nbl=4, nt=50, order=4, nshots=1, nrec=5, f_khz=0.03))
    og = c.ogrid()
    dobs = c.dobs_oracle()
    g, _ = oracle.gradient_full(og, c.m0, c.src, c.rec, c.wav, dobs)
    # histories a = u^s, b = w^s (the exact gradient is -sum_s a b); the
    # per-node variance of the r-probe estimator is
    #   (|a|^2 |b|^2 + (a.b)^2 + (kappa - 3) sum a^2 b^2) / r
    d, uh = oracle.forward(og, c.m0, c.src, c.rec, c.wav, return_history=True)
    _, lh = oracle.adjoint(og, c.m0, c.src, c.rec, d - dobs, return_history=True)
    u = uh[0].reshape(c.wl.nt, -1)
    lam = np.concatenate([lh[0].reshape(c.wl.nt, -1), np.zeros((1, u.shape[1]))])
    a, b = u[1:], lam[0:-2] - 2 * lam[1:-1] + lam[2:]
    np.testing.assert_allclose(-np.sum(a * b, axis=0), g.reshape(-1), rtol=0, atol=1e-12 * np.abs(g).max())
    r = 4
    pred = float(np.sum((np.sum(a * a, 0) * np.sum(b * b, 0) + np.sum(a * b, 0) ** 2
                         + (kappa - 3.0) * np.sum(a * a * b * b, 0)) / r))
    tg, geom, m, dd = c.tgrid(), c.tgeom(), cuda(c.m0), cuda(dobs)
    nseeds = 400
    acc = np.zeros_like(g)
    sq = 0.0
    mean_err = {}
    for s in range(nseeds):
        gp, _ = tpx.gradient_probed(tg, geom, tpx.Probe(kind=kind, r=r, seed=1000 + s), m, dd)
        gp = to_np(gp)
        acc += gp
        sq += float(np.sum((gp - g) ** 2))
        if s + 1 in (25, 100, 400):
            mean_err[s + 1] = float(np.sum((acc / (s + 1) - g) ** 2))
    ratio = (sq / nseeds) / pred
    print(f"[probe_statistics] E|g~-g|^2 / predicted = {ratio:.3f}; mean errors {mean_err}", flush=True)
    assert 0.8 < ratio < 1.25, ratio
    for n, e in mean_err.items():
        assert 0.25 < e / (pred / n) < 4.0, (n, e / (pred / n))
    assert mean_err[400] < mean_err[25] / 4.0
