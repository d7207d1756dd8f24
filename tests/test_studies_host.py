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


def test_band_basis_orthonormal_and_in_band():
    from paper_2104_00794_amd.studies import band_basis
    nt, dt, f = 400, 1.25, 0.015
    V = band_basis(nt, dt, f)
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-10
    # spectrum of every column sits on the band's DFT bins
    F = np.abs(np.fft.rfft(V, axis=0)) ** 2
    fr = np.fft.rfftfreq(nt, dt)
    inband = (fr >= 0.25 * f - 1e-12) & (fr <= 2.5 * f + 1e-12)
    assert V.shape[1] == 2 * int(inband[1:nt // 2].sum())
    assert F[~inband].sum() < 1e-20 * F.sum()


def test_outer_distance_against_dense_and_closed_forms():
    from paper_2104_00794_amd.studies import band_basis, fourier_probes, outer_distance
    rng = np.random.default_rng(3)
    nt, dt, f, r = 240, 1.25, 0.015, 8
    V = band_basis(nt, dt, f)
    nb = V.shape[1]
    # dense evaluation of both norms
    Z = rng.standard_normal((nt, r))
    M = Z @ Z.T / r - np.eye(nt)
    full, band = outer_distance(Z, 1.0 / r, V)
    assert abs(full - np.linalg.norm(M) / math.sqrt(nt)) < 1e-10 * full
    assert abs(band - np.linalg.norm(V.T @ M @ V) / math.sqrt(nb)) < 1e-10 * band
    # orthonormal columns: ||Q Q^T - I||_F^2 = n_t - r; inside the band, when Q
    # spans r of the band's own directions, n_B - r
    Q = fourier_probes(nt, dt, f, r, 1)[0].astype(np.float64)
    Q = np.linalg.qr(Q)[0]
    assert abs(outer_distance(Q, 1.0, V)[0] ** 2 - (nt - r) / nt) < 1e-10
    Qb = V[:, :r]
    assert abs(outer_distance(Qb, 1.0, V)[1] ** 2 - (nb - r) / nb) < 1e-10
    # identity probing (r = n_t, c = 1) is exact
    assert max(outer_distance(np.eye(nt), 1.0, V)) < 1e-6
    # Rademacher: the diagonal of Z Z^T / r is exactly one, the off-diagonal
    # entries have variance 1/r, so E||.||_F^2 / n_t = (n_t - 1) / r
    vals = [outer_distance(rng.choice([-1.0, 1.0], size=(nt, r)), 1.0 / r, V)[0] ** 2 for _ in range(200)]
    assert abs(np.mean(vals) - (nt - 1) / r) < 0.02 * (nt - 1) / r
