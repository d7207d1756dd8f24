"""Shared test plumbing: builds the oracle's and the GPU library's views of one
seeded workload from the same bytes (inputs rounded to float32 once, then fed
to both sides)."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2104_00794_amd.inputs import Workload  # noqa: E402


def ensure_built():
    from paper_2104_00794_amd import build as b
    if b.stale():
        b.build(force=True)
    oracle.build(force=False)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


class Case:
    """Inputs of one workload: float32-representable models and wavelets."""

    def __init__(self, wl: Workload, nt=None, shots=None):
        if nt is not None:
            wl = wl.with_(nt=nt)
        if shots is not None:
            wl = wl.with_(src=[wl.src[i] for i in shots])
        self.wl = wl
        mt, m0 = wl.models()
        self.m_true = f32(mt)
        self.m0 = f32(m0)
        self.src = wl.src_pos()
        self.rec = wl.rec_pos()
        self.wav = f32(wl.wavelet())

    def ogrid(self):
        w = self.wl
        return oracle.Grid(w.shape, h=w.h, dt=w.dt, nt=w.nt, order=w.order, nbl=w.nbl, damp_vmax=w.vmax,
                           damp_R=w.damp_R)

    def tgrid(self):
        from paper_2104_00794_amd import tpx
        w = self.wl
        return tpx.Grid(w.shape, h=w.h, dt=w.dt, nt=w.nt, order=w.order, nbl=w.nbl, damp_vmax=w.vmax,
                        damp_R=w.damp_R)

    def tgeom(self, device="cuda"):
        import torch
        from paper_2104_00794_amd import tpx
        return tpx.Geometry(self.src, self.rec, torch.tensor(self.wav, dtype=torch.float32, device=device))

    def dobs_oracle(self):
        # the oracle's traces of the true model; those of large problems (the
        # full-size configurations, minutes of FP64 work) are kept for the
        # session, keyed by the complete workload description
        big = self.m_true.size * self.wl.nt * len(self.src) > 10 ** 9
        key = repr(self.wl)
        if big and key in _DOBS:
            return _DOBS[key].copy()
        d = f32(oracle.forward(self.ogrid(), self.m_true, self.src, self.rec, self.wav))
        if big:
            _DOBS.clear()
            _DOBS[key] = d.copy()
        return d


_DOBS = {}   # observed data of the last large workload (see Case.dobs_oracle)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def cuda(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")
