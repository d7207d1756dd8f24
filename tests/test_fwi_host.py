"""CPU tests of the inversion driver's host logic (paper_2104_00794_amd/fwi.py):
the SPG loop on CPU tensors against SciPy's bounded least squares and the
closed forms of SPG on quadratics, and the seeded shot batches."""
import numpy as np
import torch
from scipy.optimize import lsq_linear

from paper_2104_00794_amd import fwi


def test_spg_bounded_least_squares_matches_scipy():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 15))
    b = rng.standard_normal(40) * 3.0
    lo, hi = -0.3, 0.4
    ref = lsq_linear(A, b, bounds=(lo, hi), tol=1e-14, lsmr_tol="auto", max_iter=10000).x
    At = torch.tensor(A)
    bt = torch.tensor(b)

    def f(x, k):
        return 0.5 * float(((At @ x - bt) ** 2).sum())

    def fg(x, k):
        r = At @ x - bt
        return 0.5 * float(r @ r), At.T @ r

    res = fwi.spg(fg, f, torch.zeros(15, dtype=torch.float64), lo, hi, fwi.SPGOptions(iters=400))
    assert np.max(np.abs(res.x.numpy() - ref)) < 1e-8


def test_spg_unit_hessian_and_interpolated_step():
    c = torch.tensor(np.random.default_rng(5).uniform(-2.0, 2.0, 50))

    def f(x, k):
        return 0.5 * float(((x - c) ** 2).sum())

    res = fwi.spg(lambda x, k: (f(x, k), x - c), f, torch.zeros(50, dtype=torch.float64), -1.0, 1.0,
                  fwi.SPGOptions(iters=2))
    assert abs(res.history[1].alpha - 1.0) < 1e-12
    assert float((res.x - c.clamp(-1.0, 1.0)).abs().max()) < 1e-12

    def f1(x, k):
        return 0.5 * float(x[0] ** 2)

    res = fwi.spg(lambda x, k: (f1(x, k), x.clone()), f1, torch.ones(1, dtype=torch.float64), -100.0, 100.0,
                  fwi.SPGOptions(iters=1, step0=5.0 / 200.0))
    h = res.history[0]
    assert h.trials == 2 and abs(h.t - 0.2) < 1e-15 and abs(float(res.x[0])) < 1e-15


def test_spg_keeps_the_model_when_no_trial_passes():
    # an objective that jumps up at every point but the start: every trial fails
    def f(x, k):
        return 1.0 if float(x.abs().max()) == 0.0 else 2.0

    res = fwi.spg(lambda x, k: (f(x, k), torch.ones_like(x)), f, torch.zeros(3, dtype=torch.float64), -1.0, 1.0,
                  fwi.SPGOptions(iters=1, max_ls=4))
    assert res.history[0].t == 0.0 and res.history[0].trials == 4
    assert float(res.x.abs().max()) == 0.0


def test_batches_are_seeded_sorted_subsets():
    a = fwi.batches(49, 20, 5, seed=7)
    b = fwi.batches(49, 20, 5, seed=7)
    assert len(a) == 5
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
        assert len(set(x.tolist())) == 20 and np.all(np.diff(x) > 0) and x.max() < 49
    assert not np.array_equal(a[0], a[1])
    assert fwi.parse_gradient("exact") == ("exact", 0)
    assert fwi.parse_gradient("gauss_b64:16") == ("gauss_b64", 16)
