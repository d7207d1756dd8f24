"""CPU tests of the seeded input generators: the named workloads have the
grid, record, acquisition and probe settings of the configurations they stand
for, fit the leapfrog stability limit, and are reproducible from their seeds."""
import math

import numpy as np
import pytest

from paper_2104_00794_amd.inputs import WORKLOADS, ricker, workload

# largest Courant numbers of the leapfrog scheme: 2 / sqrt(D sum|c|)
SUM_ABS_C = {4: 16.0 / 3.0, 8: 6.50159}


def courant(wl):
    return wl.vmax * wl.dt / wl.h


@pytest.mark.parametrize("name", WORKLOADS)
def test_within_the_stability_limit(name):
    wl = workload(name)
    limit = 2.0 / math.sqrt(wl.ndim * SUM_ABS_C[wl.order])
    assert courant(wl) <= limit
    assert wl.velocity_true().max() <= wl.vmax + 1e-12 and wl.velocity_true().min() >= wl.vmin - 1e-12


def test_c1_acquisition():
    wl = workload("c1_layered_2d_16shots")
    assert wl.shape == (301, 801) and wl.h == 12.5 and wl.order == 8 and wl.nbl == 20
    assert wl.nt == 2401 and abs((wl.nt - 1) * wl.dt - 3000.0) < 1e-9     # 3 s records
    assert wl.f_khz == 0.015 and wl.r == 16
    src = wl.src_pos()
    assert src.shape == (16, 3)
    assert np.allclose(src[:, 0], 500.0 + 600.0 * np.arange(16)) and np.all(src[:, 2] == 50.0)
    rec = wl.rec_pos()
    assert rec.shape == (16, 201, 3) and np.allclose(np.diff(rec[0, :, 0]), 50.0) and np.all(rec[..., 2] == 500.0)
    assert wl.n_pad == 841 * 341


def test_c3_acquisition():
    wl = workload("c3_layered_3d")
    assert wl.shape == (301, 401, 401) and wl.h == 12.5 and wl.nt == 2001 and wl.r == 32
    rec = wl.rec_pos()
    assert rec.shape == (1, 201 * 201, 3) and np.all(rec[..., 2] == 50.0)
    assert np.allclose(wl.src_pos(), [[2500.0, 2500.0, 50.0]])
    assert wl.n_pad == 441 * 441 * 341


def test_c0_and_c2():
    c0 = workload("c0_two_layer_2d")
    assert c0.shape == (101, 101) and c0.order == 4 and c0.nt == 501 and c0.r == 8
    v = c0.velocity_true()
    assert np.all(v[:50] == 1.5) and np.all(v[51:] == 2.5)      # the interface at 500 m depth
    c2 = workload("c2_autograd_2d")
    assert c2.shape == (201, 401) and c2.nshots == 4 and c2.r == 32 and c2.nt == 2001


def test_models_are_reproducible_and_smoothed():
    wl = workload("c1_layered_2d_16shots")
    mt1, m01 = wl.models()
    mt2, m02 = wl.models()
    assert np.array_equal(mt1, mt2) and np.array_equal(m01, m02)
    assert np.allclose(mt1, 1.0 / wl.velocity_true() ** 2)
    # the starting model is smoother than the true one
    assert np.abs(np.diff(m01, axis=0)).max() < np.abs(np.diff(mt1, axis=0)).max()


def test_ricker_peak_and_delay():
    # t0 = 1/f falls on sample 100 here: peak exactly 1, even about it, zeros at
    # tau = +-1/(sqrt(2) pi f), and below 1e-3 of the peak at t = 0
    f, dt = 0.01, 1.0
    w = ricker(f, dt, 201)
    assert w[100] == 1.0 and int(np.argmax(w)) == 100
    assert np.allclose(w[:100], w[200:100:-1], rtol=0, atol=1e-15)
    tz = 1.0 / (math.sqrt(2.0) * math.pi * f)
    assert ricker(f, tz, 2, t0=0.0)[1] == pytest.approx(0.0, abs=1e-15)
    assert abs(w[0]) < 1e-3
