"""FP64 reference of the inversion loop: spectral projected gradient (SPG)
with box constraints and random shot batches.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the plain NumPy loop
that the library's inversion driver is checked against.  It shares no code
with ``paper_2104_00794_amd`` and imports nothing from it.

The paper's inversion experiment (Example section) runs SPG, i.e. gradient
descent with box constraints, with a new random subset of shots at every
iteration.  The method is the spectral projected gradient of Birgin,
Martinez & Raydan (SIAM J. Optim. 10, 2000; "SPG2"), as packaged by Schmidt
et al. (2009), which the paper cites.  Each iteration here:

  1. evaluates f_k and g_k on the iteration's batch at x_k;
  2. takes the spectral (Barzilai-Borwein) step a_k = s's / s'y from the last
     move s = x_k - x_{k-1} and gradient change y = g_k - g_{k-1}, or a_max
     when s'y <= 0, clipped to [a_min, a_max]; the first step is chosen so
     that the largest entry of a_0 g_0 equals `step0` times the widest bound
     interval;
  3. forms the projected direction d_k = P(x_k - a_k g_k) - x_k, with P the
     projection onto the box lo <= x <= hi;
  4. backtracks along d_k from t = 1 until the Armijo condition
     f(x_k + t d_k) <= f_k + gamma t g_k'd_k holds on the same batch, each new
     t the minimiser of the quadratic through f_k, g_k'd_k and the last trial,
     kept within [sigma1 t, sigma2 t] (else t / 2);
  5. moves to x_{k+1} = x_k + t d_k, or stays at x_k when `max_ls` trials fail.

With one batch (a deterministic objective) and memory one in the
non-monotone test this is SPG2 as published; the safeguards a_min, a_max are
relative to the first step, because the objective's scale is arbitrary.

Parity status: pinned by tests/test_oracle_spg.py against SciPy's bounded
least-squares solver and against closed forms of SPG on separable quadratics.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


@dataclass
class Options:
    iters: int = 20
    step0: float = 0.02
    gamma: float = 1e-4
    sigma1: float = 0.1
    sigma2: float = 0.9
    max_ls: int = 10
    alpha_range: float = 1e3


@dataclass
class Record:
    f: float           # objective at x_k on batch k
    gnorm: float       # max |g_k|
    alpha: float       # spectral step a_k
    t: float           # accepted line-search fraction (0 when no trial passed)
    trials: int        # objective evaluations of the line search
    f_new: float       # objective at x_{k+1} on batch k


@dataclass
class Result:
    x: np.ndarray
    history: List[Record] = field(default_factory=list)


def project(x, lo, hi):
    """Closest point of the box lo <= x <= hi (lo, hi scalars or arrays)."""
    return np.minimum(np.maximum(x, lo), hi)


def spg(fg: Callable, f: Callable, x0, lo, hi, opts: Options = Options()) -> Result:
    """Minimise over the box.  fg(x, k) -> (f, g) and f(x, k) -> f evaluate the
    objective (and gradient) of iteration k's batch at x."""
    x = project(np.asarray(x0, dtype=np.float64), lo, hi)
    width = float(np.max(np.broadcast_to(np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64),
                                          x.shape)))
    out = Result(x=x)
    x_prev = g_prev = None
    a_min = a_max = None
    for k in range(opts.iters):
        fk, gk = fg(x, k)
        gk = np.asarray(gk, dtype=np.float64)
        gmax = float(np.max(np.abs(gk)))
        if k == 0:
            a0 = opts.step0 * width / gmax if gmax > 0 else 1.0
            a_min, a_max = a0 / opts.alpha_range, a0 * opts.alpha_range
            alpha = a0
        else:
            s = x - x_prev
            y = gk - g_prev
            sy = float(np.sum(s * y))
            alpha = a_max if sy <= 0 else min(max(float(np.sum(s * s)) / sy, a_min), a_max)
        d = project(x - alpha * gk, lo, hi) - x
        slope = float(np.sum(gk * d))
        t, trials, accepted, f_new = 1.0, 0, False, fk
        if slope < 0:
            while trials < opts.max_ls:
                ft = float(f(x + t * d, k))
                trials += 1
                if ft <= fk + opts.gamma * t * slope:
                    accepted, f_new = True, ft
                    break
                # minimiser of q(s) = fk + slope s + c s^2 through (t, ft)
                c = (ft - fk - slope * t) / (t * t)
                t_q = -slope / (2.0 * c)
                t = t_q if opts.sigma1 * t <= t_q <= opts.sigma2 * t else 0.5 * t
        x_prev, g_prev = x, gk
        if accepted:
            x = x + t * d
        out.history.append(Record(f=float(fk), gnorm=gmax, alpha=float(alpha), t=t if accepted else 0.0,
                                  trials=trials, f_new=float(f_new)))
    out.x = x
    return out
