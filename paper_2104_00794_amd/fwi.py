"""Full-waveform inversion driven by the probed gradient (Example section).

The paper inverts for squared slowness with spectral projected gradient (SPG:
gradient descent with box constraints, Birgin, Martinez & Raydan 2000, as
packaged by Schmidt et al. 2009) and a new random subset of shots at every
iteration.  This module runs that loop on one GPU:

* the gradient of each iteration's batch comes from ``tpx_gradient_probed``
  (Eq. 4, Algorithm 1) or, for comparison, ``tpx_gradient_full`` (Eq. 3);
* the line search evaluates the batch objective with ``tpx_objective``
  (Eq. 2), forward modelling only;
* the optimiser's own vector work (a projection, two axpys and three dot
  products per iteration, O(N) against the O(N n_t S) of a gradient) runs as
  device tensor operations.

One iteration: the spectral step a_k = s's / s'y (a_max when s'y <= 0, clipped
to [a_0 / 1e3, a_0 * 1e3]; a_0 moves the largest model entry by `step0` times
the widest bound interval), the projected direction d_k = P(x_k - a_k g_k) -
x_k, and an Armijo backtracking search along d_k on the same batch with
safeguarded quadratic interpolation.  A search with no acceptable trial leaves
the model unchanged.

    python -m paper_2104_00794_amd.fwi --workload f4_fwi_2d --gradient exact rademacher:16
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import tpx
from .inputs import Workload, workload


@dataclass
class SPGOptions:
    iters: int = 20
    step0: float = 0.02       # first move, as a fraction of the widest bound interval
    gamma: float = 1e-4       # sufficient-decrease constant
    sigma1: float = 0.1       # quadratic-interpolation safeguards
    sigma2: float = 0.9
    max_ls: int = 10          # objective evaluations per line search
    alpha_range: float = 1e3  # spectral step kept within a_0 / range .. a_0 * range


@dataclass
class SPGStep:
    f: float
    gnorm: float
    alpha: float
    t: float
    trials: int
    f_new: float
    seconds: float = 0.0
    model_error: Optional[float] = None


@dataclass
class SPGResult:
    x: object
    history: List[SPGStep] = field(default_factory=list)


def _dot(a, b) -> float:
    return float((a.double() * b.double()).sum().item())


def spg(fg: Callable, f: Callable, x0, lo, hi, opts: SPGOptions = SPGOptions(),
        monitor: Optional[Callable] = None) -> SPGResult:
    """Box-constrained SPG on torch tensors (any device).

    fg(x, k) -> (f, g) and f(x, k) -> f evaluate iteration k's batch objective
    at x (f as a Python float, g a tensor shaped like x).  lo, hi: scalars or
    tensors shaped like x.  monitor(x, k), if given, is recorded as the
    iteration's model error after its move."""
    import torch

    def box(v):
        return torch.minimum(torch.maximum(v, lo_t), hi_t)

    lo_t = torch.as_tensor(lo, dtype=x0.dtype, device=x0.device)
    hi_t = torch.as_tensor(hi, dtype=x0.dtype, device=x0.device)
    width = float(torch.broadcast_to(hi_t - lo_t, x0.shape).max().item())
    x = box(x0.clone())
    res = SPGResult(x=x)
    prev = None   # (x, g) of the previous iteration
    a_lo = a_hi = None
    for k in range(opts.iters):
        t0 = time.perf_counter()
        fk, gk = fg(x, k)
        fk = float(fk)
        gmax = float(gk.abs().max().item())
        if prev is None:
            alpha = opts.step0 * width / gmax if gmax > 0 else 1.0
            a_lo, a_hi = alpha / opts.alpha_range, alpha * opts.alpha_range
        else:
            s, y = x - prev[0], gk - prev[1]
            sy = _dot(s, y)
            alpha = a_hi if sy <= 0 else min(max(_dot(s, s) / sy, a_lo), a_hi)
        d = box(x - alpha * gk) - x
        slope = _dot(gk, d)
        step, trials, f_new, ok = 1.0, 0, fk, False
        while slope < 0 and trials < opts.max_ls:
            f_try = float(f(x + step * d, k))
            trials += 1
            if f_try <= fk + opts.gamma * step * slope:
                ok, f_new = True, f_try
                break
            curv = (f_try - fk - slope * step) / (step * step)
            t_q = -slope / (2.0 * curv)
            step = t_q if opts.sigma1 * step <= t_q <= opts.sigma2 * step else 0.5 * step
        prev = (x, gk)
        if ok:
            x = x + step * d
        rec = SPGStep(f=fk, gnorm=gmax, alpha=float(alpha), t=step if ok else 0.0, trials=trials, f_new=f_new)
        if monitor is not None:
            rec.model_error = float(monitor(x, k))
        rec.seconds = time.perf_counter() - t0
        res.history.append(rec)
    res.x = x
    return res


# --------------------------------------------------------------------------- #
# the inversion experiment on a synthetic workload
# --------------------------------------------------------------------------- #

def batches(nshots: int, batch: int, iters: int, seed: int) -> List[np.ndarray]:
    """The shots of each iteration: a sorted random subset, drawn from a seeded generator."""
    rng = np.random.default_rng(seed)
    return [np.sort(rng.choice(nshots, size=min(batch, nshots), replace=False)) for _ in range(iters)]


def parse_gradient(spec: str):
    """'exact' or 'KIND:R' (KIND a probe kind of the library)."""
    if spec == "exact":
        return ("exact", 0)
    kind, r = spec.split(":")
    if kind not in tpx.PROBE_KINDS:
        raise ValueError("unknown probe kind %r" % kind)
    return (kind, int(r))


class Problem:
    """A workload's grid, all shots' geometry and observed data on the device."""

    def __init__(self, wl: Workload, device="cuda", chunk: int = 16):
        import torch
        self.wl = wl
        self.device = device
        self.grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl,
                             damp_vmax=wl.vmax, damp_R=wl.damp_R)
        mt, m0 = wl.models()
        self.m_true = torch.tensor(mt, dtype=torch.float32, device=device)
        self.m0 = torch.tensor(m0, dtype=torch.float32, device=device)
        self.src = wl.src_pos()
        self.rec = wl.rec_pos()
        self.wav = torch.tensor(wl.wavelet(), dtype=torch.float32, device=device)
        self.lo = 1.0 / (wl.vmax * wl.vmax)
        self.hi = 1.0 / (wl.vmin * wl.vmin)
        parts = []
        for a in range(0, wl.nshots, chunk):
            idx = np.arange(a, min(a + chunk, wl.nshots))
            parts.append(tpx.forward(self.grid, self.geometry(idx), self.m_true))
        self.d_obs = torch.cat(parts, 0)

    def geometry(self, idx) -> tpx.Geometry:
        import torch
        sel = torch.as_tensor(np.asarray(idx), dtype=torch.long, device=self.wav.device)
        return tpx.Geometry(self.src[idx], self.rec[idx], self.wav.index_select(0, sel).contiguous())

    def data(self, idx):
        import torch
        sel = torch.as_tensor(np.asarray(idx), dtype=torch.long, device=self.d_obs.device)
        return self.d_obs.index_select(0, sel).contiguous()

    def model_error(self, m) -> float:
        """||m - m_true|| / ||m0 - m_true|| over the physical grid."""
        import torch
        num = torch.linalg.vector_norm((m - self.m_true).double()).item()
        den = torch.linalg.vector_norm((self.m0 - self.m_true).double()).item()
        return num / den


def invert(prob: Problem, gradient: str, opts: SPGOptions, batch: int, batch_seed: int, probe_seed: int,
           on_step: Optional[Callable] = None):
    """One SPG inversion with the given gradient ('exact' or 'KIND:R')."""
    kind, r = parse_gradient(gradient)
    plan = batches(prob.wl.nshots, batch, opts.iters, batch_seed)
    counters = {"gradient_s": 0.0, "objective_s": 0.0, "gradients": 0, "objectives": 0}

    def sync():
        import torch
        torch.cuda.synchronize()

    def fg(x, k):
        idx = plan[k]
        geom, dobs = prob.geometry(idx), prob.data(idx)
        t0 = time.perf_counter()
        if kind == "exact":
            g, J = tpx.gradient_full(prob.grid, geom, x, dobs)
        else:
            g, J = tpx.gradient_probed(prob.grid, geom, tpx.Probe(kind=kind, r=r, seed=probe_seed + k), x, dobs)
        Jv = float(J.item())
        sync()
        counters["gradient_s"] += time.perf_counter() - t0
        counters["gradients"] += 1
        return Jv, g

    def fval(x, k):
        idx = plan[k]
        t0 = time.perf_counter()
        Jv = float(tpx.objective(prob.grid, prob.geometry(idx), x, prob.data(idx)).item())
        counters["objective_s"] += time.perf_counter() - t0
        counters["objectives"] += 1
        return Jv

    def monitor(x, k):
        err = prob.model_error(x)
        if on_step is not None:
            on_step(k, err)
        return err

    res = spg(fg, fval, prob.m0, prob.lo, prob.hi, opts, monitor=monitor)
    return res, counters


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="f4_fwi_2d")
    ap.add_argument("--gradient", nargs="+", default=["exact", "rademacher:4", "rademacher:16", "rademacher:64"])
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--batch", type=int, default=20)
    ap.add_argument("--batch-seed", type=int, default=7)
    ap.add_argument("--step0", type=float, default=SPGOptions.step0)
    ap.add_argument("--out", default=None, help="write all histories as JSON")
    a = ap.parse_args(argv)
    wl = workload(a.workload)
    t0 = time.perf_counter()
    prob = Problem(wl)
    print(json.dumps({"workload": wl.name, "shots": wl.nshots, "nt": wl.nt, "shape": list(wl.shape),
                      "observed_data_s": round(time.perf_counter() - t0, 2)}), flush=True)
    runs = []
    for spec in a.gradient:
        opts = SPGOptions(iters=a.iters, step0=a.step0)
        t1 = time.perf_counter()
        res, cnt = invert(prob, spec, opts, a.batch, a.batch_seed, wl.probe_seed,
                          on_step=lambda k, e, s=spec: print(json.dumps({"gradient": s, "iter": k,
                                                                         "model_error": round(e, 5)}), flush=True))
        secs = time.perf_counter() - t1
        nb = min(a.batch, wl.nshots)
        work = nb * float(np.prod([s + 2 * wl.nbl for s in wl.shape])) * 2 * (wl.nt - 1) * cnt["gradients"]
        row = {"gradient": spec, "iters": a.iters, "batch": nb, "seconds": round(secs, 2),
               "final_model_error": round(res.history[-1].model_error, 5),
               "f_first": res.history[0].f, "f_last": res.history[-1].f_new,
               "objective_calls": cnt["objectives"],
               "gradient_GPts_per_s": round(work / cnt["gradient_s"] / 1e9, 1),
               "history": [s.__dict__ for s in res.history]}
        runs.append(row)
        print(json.dumps({k: v for k, v in row.items() if k != "history"}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"workload": wl.name, "runs": runs}, f, indent=1)


if __name__ == "__main__":
    main()
