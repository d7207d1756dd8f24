"""CPU tests of the probe-family study's host part: the restricted Fourier
probing basis is orthonormal, shared by the shots, and spans the sinusoids of
its frequencies."""
import math

import numpy as np

from paper_2104_00794_amd.studies import fourier_probes


def test_fourier_probes_orthonormal_and_shared():
    nt, dt, f, r, S = 600, 1.25, 0.015, 16, 3
    Q = fourier_probes(nt, dt, f, r, S).astype(np.float64)
    assert Q.shape == (S, nt, r)
    assert np.array_equal(Q[0], Q[2])
    assert np.abs(Q[0].T @ Q[0] - np.eye(r)).max() < 1e-5


def test_fourier_probes_span_their_band():
    nt, dt, f, r = 600, 1.25, 0.015, 16
    Q = fourier_probes(nt, dt, f, r, 1)[0].astype(np.float64)
    t = np.arange(nt) * dt
    for fk in np.linspace(0.25 * f, 2.5 * f, r // 2):
        for v in (np.cos(2 * math.pi * fk * t), np.sin(2 * math.pi * fk * t)):
            res = v - Q @ (Q.T @ v)
            assert np.linalg.norm(res) <= 1e-5 * np.linalg.norm(v)
    # a frequency far outside the band is mostly not captured
    v = np.cos(2 * math.pi * 10 * f * t)
    assert np.linalg.norm(Q.T @ v) < 0.5 * np.linalg.norm(v)
