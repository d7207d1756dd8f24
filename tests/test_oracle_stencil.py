"""Pins of the oracle's spatial operator, model padding and absorbing layer.

None of these re-types the oracle's formulas: they check properties that the
centred second-difference stencil of a given order must have (exactness on
polynomials, the Nyquist symbol, convergence order) and behaviour of the
absorbing layer against a reflection-free reference run.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid


def _coords(grid, axis_len):
    return (np.arange(axis_len) - axis_len // 2) * grid.h


@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("ndim", [2, 3])
def test_laplacian_exact_on_polynomials(order, ndim):
    # A centred stencil of order p is exact for polynomials of degree <= p + 1.
    shape = (21, 23) if ndim == 2 else (15, 16, 17)
    grid = Grid(shape, h=0.5, dt=1.0, nt=2, order=order, nbl=0)
    P = grid.padded_shape
    R = order // 2
    axes = [np.arange(n) - n // 2 for n in P]
    for deg in range(0, order + 2):
        coef = np.random.default_rng(deg).normal(size=ndim)
        mesh = np.meshgrid(*[a * grid.h for a in axes], indexing="ij")
        u = sum(c * x ** deg for c, x in zip(coef, mesh))
        exact = sum(c * deg * (deg - 1) * x ** max(deg - 2, 0) for c, x in zip(coef, mesh)) if deg >= 2 \
            else np.zeros(P)
        Lu = oracle.laplacian(grid, u)
        inner = tuple(slice(R, n - R) for n in P)
        scale = max(np.abs(exact[inner]).max(), np.abs(u[inner]).max() / grid.h ** 2, 1.0)
        assert np.abs(Lu[inner] - exact[inner]).max() <= 1e-11 * scale, deg


@pytest.mark.parametrize("order,symbol", [(4, 16.0 / 3.0), (8, 6.501587301587302)])
def test_laplacian_nyquist_symbol(order, symbol):
    # On the checkerboard (-1)^i the centred stencil returns -sum|c| / h^2 times u.
    grid = Grid((11, 31), h=2.0, dt=1.0, nt=2, order=order, nbl=0)
    nz, nx = grid.padded_shape
    u = np.tile((-1.0) ** np.arange(nx), (nz, 1))
    Lu = oracle.laplacian(grid, u)
    R = order // 2
    inner = (slice(R, nz - R), slice(R, nx - R))
    # the z-direction sees a constant in z, which the stencil annihilates
    np.testing.assert_allclose(Lu[inner], -symbol / grid.h ** 2 * u[inner], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("order", [4, 8])
def test_laplacian_convergence_order(order):
    # Error on sin(k x) falls like h^order.
    errs = []
    for n in (33, 65):
        L = 1.0
        h = L / (n - 1)
        grid = Grid((9, n), h=h, dt=1.0, nt=2, order=order, nbl=0)
        x = np.arange(n) * h
        k = 2 * np.pi * 3
        u = np.tile(np.sin(k * x), (9, 1))
        Lu = oracle.laplacian(grid, u)
        R = order // 2
        inner = (slice(R, 9 - R), slice(3 * R, n - 3 * R))
        errs.append(np.abs(Lu[inner] + k * k * u[inner]).max())
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - order) < 0.35, (errs, rate)


def test_pad_model_is_edge_replication():
    rng = np.random.default_rng(0)
    for shape, nbl in (((7, 9), 3), ((4, 5, 6), 2)):
        m = rng.uniform(0.1, 0.5, size=shape)
        grid = Grid(shape, h=1.0, dt=1.0, nt=2, order=4, nbl=nbl)
        np.testing.assert_array_equal(oracle.pad_model(grid, m), np.pad(m, nbl, mode="edge"))


def test_damping_zero_inside_and_growing_outward():
    grid = Grid((12, 14), h=10.0, dt=1.0, nt=2, order=8, nbl=6, damp_vmax=3.0)
    d = oracle.damping(grid)
    nb = grid.nbl
    assert np.all(d[nb:-nb, nb:-nb] == 0.0)
    assert np.all(d >= 0.0)
    row = d[nb + 5, :nb + 1]
    assert np.all(np.diff(row) < 0)           # decreasing towards the physical region
    corner = d[0, 0]
    assert corner == pytest.approx(2 * d[0, nb + 5])  # two axes add at the corner


def _homogeneous_trace(nphys, nbl, damp_R, nt=260):
    v = 2.0
    h = 10.0
    dt = 0.8 * 0.5546 * h / v
    grid = Grid((nphys, nphys), h=h, dt=dt, nt=nt, order=8, nbl=nbl, damp_vmax=v, damp_R=damp_R)
    m = np.full((nphys, nphys), 1.0 / v ** 2)
    c = (nphys - 1) * h / 2
    src = np.array([[c, 0.0, c]])
    rec = np.array([[[c + 60.0, 0.0, c]]])
    from paper_2104_00794_amd.inputs import ricker
    w = ricker(0.02, dt, nt)[None, :]
    return oracle.forward(grid, m, src, rec, w)[0, :, 0]


def test_absorbing_layer_removes_boundary_reflection():
    # Reference: a box large enough that nothing comes back within the record.
    ref = _homogeneous_trace(301, 0, 1.0)
    small = _homogeneous_trace(41, 20, 1e-3)
    rigid = _homogeneous_trace(41, 20, 1.0)   # R = 1 switches the damping off
    e_ref = np.sum(ref ** 2)
    refl_damped = np.sum((small - ref) ** 2) / e_ref
    refl_rigid = np.sum((rigid - ref) ** 2) / e_ref
    assert refl_rigid > 0.1
    assert refl_damped < 0.02 * refl_rigid


def test_damping_strength_gives_round_trip_amplitude_sqrt_R():
    # A plane wave in m u_tt + m d u_t = Lap u decays as exp(-d x / (2 v)) when
    # d << omega, so a round trip through the layer (d = dmax (x/L)^2) keeps
    # exp(-dmax L / (3 v)) of its amplitude: sqrt(R) for dmax = 3 v ln(1/R) / (2 L).
    # While damping is weak the reflection off the layer is that round trip,
    # so its amplitude scales as R^(1/2); a dmax off by a factor 2 gives R or R^(1/4).
    ref = _homogeneous_trace(301, 0, 1.0)
    rigid = np.sqrt(np.sum((_homogeneous_trace(41, 20, 1.0) - ref) ** 2))
    amp = {R: np.sqrt(np.sum((_homogeneous_trace(41, 20, R) - ref) ** 2)) / rigid for R in (0.3, 0.1, 0.01)}
    for lo, hi in ((0.1, 0.3), (0.01, 0.1)):
        slope = np.log(amp[hi] / amp[lo]) / np.log(hi / lo)
        assert 0.4 < slope < 0.6, (lo, hi, slope)
