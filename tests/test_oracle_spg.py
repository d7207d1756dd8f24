"""Pins of the oracle's inversion loop (oracle/spg.py): spectral projected
gradient with box constraints (Example section; Birgin, Martinez & Raydan
2000).  Checked against SciPy's bounded least-squares solver and against
closed forms of SPG on quadratics, never against itself."""
import numpy as np
from scipy.optimize import lsq_linear

from oracle import spg as ospg


def _lsq_problem(seed=3, m=40, n=15):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m) * 3.0
    lo, hi = -0.3 * np.ones(n), 0.4 * np.ones(n)
    return A, b, lo, hi


def test_bounded_least_squares_matches_scipy():
    A, b, lo, hi = _lsq_problem()
    ref = lsq_linear(A, b, bounds=(lo, hi), tol=1e-14, lsmr_tol="auto", max_iter=10000).x
    assert np.sum((ref <= lo + 1e-9) | (ref >= hi - 1e-9)) >= 3   # several bounds active

    def f(x, k):
        return 0.5 * float(np.sum((A @ x - b) ** 2))

    def fg(x, k):
        r = A @ x - b
        return 0.5 * float(r @ r), A.T @ r

    res = ospg.spg(fg, f, np.zeros(A.shape[1]), lo, hi, ospg.Options(iters=400))
    assert np.max(np.abs(res.x - ref)) < 1e-8
    assert np.all(res.x >= lo) and np.all(res.x <= hi)
    fs = [h.f for h in res.history]
    assert all(b_ <= a_ + 1e-12 for a_, b_ in zip(fs, fs[1:]))   # monotone on one batch


def test_unit_hessian_reaches_the_projection_in_two_iterations():
    # f = 1/2 ||x - c||^2: the spectral step is exactly 1 after the first move,
    # so the second iterate is P(c), the constrained minimiser.
    rng = np.random.default_rng(5)
    c = rng.uniform(-2.0, 2.0, 50)

    def f(x, k):
        return 0.5 * float(np.sum((x - c) ** 2))

    def fg(x, k):
        return f(x, k), x - c

    res = ospg.spg(fg, f, np.zeros(50), -1.0, 1.0, ospg.Options(iters=2))
    assert res.history[0].t == 1.0 and res.history[0].trials == 1
    assert abs(res.history[0].alpha - 0.02 * 2.0 / np.max(np.abs(c))) < 1e-15
    assert abs(res.history[1].alpha - 1.0) < 1e-12
    assert np.max(np.abs(res.x - np.clip(c, -1.0, 1.0))) < 1e-12


def test_quadratic_interpolation_finds_the_exact_minimiser():
    # f = 1/2 x^2 from x0 = 1 with a first step of 5: the unit trial overshoots
    # to -4 (f = 8); the quadratic through f(0) = 1/2, f'(0) = -5 and f(1) = 8
    # has its minimiser at t = 0.2, which is x = 0.
    def f(x, k):
        return 0.5 * float(x[0] ** 2)

    def fg(x, k):
        return f(x, k), np.array([x[0]])

    res = ospg.spg(fg, f, np.array([1.0]), -100.0, 100.0, ospg.Options(iters=1, step0=5.0 / 200.0))
    h = res.history[0]
    assert h.trials == 2 and abs(h.t - 0.2) < 1e-15 and abs(res.x[0]) < 1e-15 and h.f_new == 0.0


def test_batches_change_the_objective_between_iterations():
    # Two alternating quadratics with a common box-constrained minimiser:
    # each iteration's line search uses its own batch, and the iterates still
    # converge to that minimiser.
    c = np.array([0.5, -2.0, 3.0, -0.25])
    W = [np.array([1.0, 2.0, 0.5, 1.5]), np.array([2.0, 0.7, 1.3, 0.9])]

    def f(x, k):
        return 0.5 * float(np.sum(W[k % 2] * (x - c) ** 2))

    def fg(x, k):
        return f(x, k), W[k % 2] * (x - c)

    res = ospg.spg(fg, f, np.zeros(4), -1.0, 1.0, ospg.Options(iters=60))
    assert np.max(np.abs(res.x - np.clip(c, -1.0, 1.0))) < 1e-10
