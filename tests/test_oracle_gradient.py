"""Pins of the oracle's exact and probed gradients.

* Taylor test: J(m + h dm) - J(m) - h <g, dm> = O(h^2);
* brute-force central finite differences of J on every interior cell;
* the two summation-by-parts forms of Eq. (3) agree;
* probed gradient with the identity (r = n_t) or any complete orthonormal
  basis recovers the exact gradient; it is invariant under Z -> Z O;
* unbiasedness and the closed-form variance of the Hutchinson estimator,
  E||g~ - g||^2 = sum_x Var_x with
  Var_x = (1/r) (|a|^2 |b|^2 + (a.b)^2 + (kappa - 3) sum a_t^2 b_t^2),
  a = u(x, .), b = w(x, .) and kappa the fourth moment of the probe entries;
* the probed gradient is quadratic in the source amplitude.
"""
import numpy as np
import pytest
from scipy.fft import dct
from scipy.stats import ortho_group

import oracle
from oracle import Grid
from paper_2104_00794_amd.inputs import small_2d, small_3d


def _setup(wl):
    mt, m0 = wl.models()
    grid = Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
    dobs = oracle.forward(grid, mt, wl.src_pos(), wl.rec_pos(), wl.wavelet())
    return grid, mt, m0, dobs


def _J(grid, wl, m, dobs):
    d = oracle.forward(grid, m, wl.src_pos(), wl.rec_pos(), wl.wavelet())
    return 0.5 * float(np.sum((d - dobs) ** 2))


def _edge_free(a):
    b = np.array(a, copy=True)
    if b.ndim == 2:
        b[0, :] = b[-1, :] = 0
        b[:, 0] = b[:, -1] = 0
    else:
        b[0] = b[-1] = 0
        b[:, 0] = b[:, -1] = 0
        b[:, :, 0] = b[:, :, -1] = 0
    return b


@pytest.mark.parametrize("ndim", [2, 3])
def test_taylor_second_order(ndim):
    wl = small_2d(nt=220) if ndim == 2 else small_3d(nt=80)
    grid, mt, m0, dobs = _setup(wl)
    g, J0 = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs)
    assert J0 == pytest.approx(_J(grid, wl, m0, dobs), rel=1e-12)
    dm = _edge_free(mt - m0)
    gdm = float(np.sum(g * dm))
    # h = 0.1 ... 9.8e-5, halving: in FP64 the first-order remainder halves and
    # the second-order one quarters all the way down (ratios 2.000 and 4.000
    # from h = 2.5e-2 on; the smallest second-order remainder is ~1e-8 J0)
    hs = [0.1 / 2 ** i for i in range(11)]
    r1, r2 = [], []
    for h in hs:
        Jh = _J(grid, wl, m0 + h * dm, dobs)
        r1.append(abs(Jh - J0))
        r2.append(abs(Jh - J0 - h * gdm))
    q1 = [r1[i] / r1[i + 1] for i in range(len(hs) - 1)]
    q2 = [r2[i] / r2[i + 1] for i in range(len(hs) - 1)]
    assert hs[-1] < 1e-4
    assert all(1.9 < q < 2.1 for q in q1), q1
    assert all(3.9 < q < 4.1 for q in q2), q2
    assert all(abs(q - 4.0) < 0.01 for q in q2[3:]), q2


@pytest.mark.parametrize("order", [4, 8])
def test_bruteforce_finite_differences_every_interior_cell(order):
    wl = small_2d(nz=10, nx=10, nbl=4, nt=60, order=order, nshots=1, nrec=4, f_khz=0.03)
    grid, mt, m0, dobs = _setup(wl)
    g, _ = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs)
    fd = np.zeros_like(g)
    for iz in range(1, 9):
        for ix in range(1, 9):
            eps = 1e-4 * m0[iz, ix]
            mp = m0.copy(); mp[iz, ix] += eps
            mm = m0.copy(); mm[iz, ix] -= eps
            fd[iz, ix] = (_J(grid, wl, mp, dobs) - _J(grid, wl, mm, dobs)) / (2 * eps)
    inner = (slice(1, 9), slice(1, 9))
    err = np.abs(fd[inner] - g[inner])
    assert err.max() <= 1e-6 * np.abs(g[inner]).max(), err.max() / np.abs(g[inner]).max()


def test_two_summation_forms_agree():
    wl = small_2d(nt=200)
    grid, mt, m0, dobs = _setup(wl)
    g0, J0 = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, form=0)
    g1, J1 = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, form=1)
    assert J0 == J1
    assert np.abs(g0 - g1).max() <= 1e-13 * np.abs(g0).max()


@pytest.mark.parametrize("side", [0, 1])
def test_identity_probes_recover_exact_gradient(side):
    wl = small_2d(nt=150)
    grid, mt, m0, dobs = _setup(wl)
    g, J = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs)
    gp, Jp = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs,
                                    kind="identity", r=wl.nt, side=side)
    assert Jp == J
    assert np.abs(gp - g).max() <= 1e-12 * np.abs(g).max()


def test_orthonormal_dct_basis_recovers_exact_gradient():
    wl = small_2d(nt=120, nshots=1)
    grid, mt, m0, dobs = _setup(wl)
    g, _ = oracle.gradient_full(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs)
    Q = dct(np.eye(wl.nt), norm="ortho", axis=0)   # orthonormal DCT-II, complete basis
    gp, _ = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs,
                                   kind="explicit", r=wl.nt, Z=Q[None], scale=1.0)
    assert np.abs(gp - g).max() <= 1e-12 * np.abs(g).max()


def test_probed_gradient_invariant_under_orthogonal_mixing():
    wl = small_2d(nt=100, nshots=1)
    grid, mt, m0, dobs = _setup(wl)
    rng = np.random.default_rng(9)
    r = 6
    Z = rng.normal(size=(wl.nt, r))
    O = ortho_group.rvs(r, random_state=4)
    kw = dict(kind="explicit", r=r, scale=1.0 / r)
    ga, _ = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, Z=Z[None], **kw)
    gb, _ = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, Z=(Z @ O)[None], **kw)
    gc, _ = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs,
                                   Z=Z[:, ::-1].copy()[None], **kw)
    assert np.abs(ga - gb).max() <= 1e-12 * np.abs(ga).max()
    assert np.abs(ga - gc).max() <= 1e-13 * np.abs(ga).max()


def test_points_subset_matches_full_array():
    wl = small_2d(nt=90)
    grid, mt, m0, dobs = _setup(wl)
    full, J = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, r=5, seed=3)
    pts = np.array([0, 17, 333, full.size - 1, 805])
    sub, Js = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), dobs, r=5, seed=3,
                                     points=pts)
    assert J == Js
    np.testing.assert_array_equal(sub, full.reshape(-1)[pts])


def test_probed_gradient_quadratic_in_source_amplitude():
    wl = small_2d(nt=100)
    grid, mt, m0, _ = _setup(wl)
    zero = np.zeros((wl.nshots, wl.nt, len(wl.rec)))
    g1, J1 = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), wl.wavelet(), zero, r=4, seed=5)
    g3, J3 = oracle.gradient_probed(grid, m0, wl.src_pos(), wl.rec_pos(), 3.0 * wl.wavelet(), zero, r=4, seed=5)
    assert np.abs(g3 - 9.0 * g1).max() <= 1e-12 * np.abs(g3).max()
    assert J3 == pytest.approx(9.0 * J1, rel=1e-13)


@pytest.mark.parametrize("kind,kappa", [("rademacher", 1.0), ("gauss_b64", 3.0 - 2.0 / 64.0)])
def test_unbiased_with_closed_form_variance(kind, kappa):
    wl = small_2d(nz=16, nx=18, nbl=4, nt=50, order=4, nshots=1, nrec=5, f_khz=0.03)
    grid, mt, m0, dobs = _setup(wl)
    src, rec, wav = wl.src_pos(), wl.rec_pos(), wl.wavelet()
    g, J = oracle.gradient_full(grid, m0, src, rec, wav, dobs)
    # histories a = u^s, b = w^s = lam^{s-1} - 2 lam^s + lam^{s+1}, s = 1..nt-1
    d, uh = oracle.forward(grid, m0, src, rec, wav, return_history=True)
    _, lh = oracle.adjoint(grid, m0, src, rec, d - dobs, return_history=True)
    u = uh[0].reshape(wl.nt, -1)
    lam = np.concatenate([lh[0].reshape(wl.nt, -1), np.zeros((1, u.shape[1]))])
    a = u[1:]
    b = lam[0:-2] - 2 * lam[1:-1] + lam[2:]
    # the histories reproduce the exact gradient (closed-form check of the pieces)
    np.testing.assert_allclose(-np.sum(a * b, axis=0), g.reshape(-1), rtol=0, atol=1e-12 * np.abs(g).max())
    r = 4
    var = (np.sum(a * a, 0) * np.sum(b * b, 0) + np.sum(a * b, 0) ** 2
           + (kappa - 3.0) * np.sum(a * a * b * b, 0)) / r
    pred = float(np.sum(var))
    nseeds = 300
    acc = np.zeros_like(g)
    sq = 0.0
    for s in range(nseeds):
        gp, _ = oracle.gradient_probed(grid, m0, src, rec, wav, dobs, kind=kind, r=r, seed=1000 + s)
        acc += gp
        sq += float(np.sum((gp - g) ** 2))
    assert 0.8 < (sq / nseeds) / pred < 1.25, (sq / nseeds) / pred
    mean_err = float(np.sum((acc / nseeds - g) ** 2))
    assert 0.25 < mean_err / (pred / nseeds) < 4.0, mean_err / (pred / nseeds)


# --------------------------------------------------------------------------- #
# imaging conditions on the probed fields (Eq. 5)
# --------------------------------------------------------------------------- #

def _grad_dot(h, A, B):
    """Centred-difference gradient inner product over the last 2 (2D) or 3 (3D)
    axes, zero on the outermost nodes; written with array slices."""
    nd = A.ndim - 1
    out = np.zeros(A.shape)
    inner = (slice(None),) + (slice(1, -1),) * nd
    for ax in range(1, nd + 1):
        hi = list(inner)
        lo = list(inner)
        hi[ax] = slice(2, None)
        lo[ax] = slice(None, -2)
        out[inner] += ((A[tuple(hi)] - A[tuple(lo)]) / (2 * h)) * ((B[tuple(hi)] - B[tuple(lo)]) / (2 * h))
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_imaging_commutes_with_probing(ndim):
    # Eq. 5: a space-only linear operator (here grad) applied to the r probed
    # fields equals probing the operator applied to every snapshot
    if ndim == 2:
        wl = small_2d(nz=14, nx=17, nbl=4, nt=40, order=4, nshots=1, nrec=5)
    else:
        wl = small_3d(nz=10, ny=7, nx=9, nbl=3, nt=30, order=4, nshots=1, nrec=4)
    grid, mt, m0, dobs = _setup(wl)
    src, rec, wav = wl.src_pos(), wl.rec_pos(), wl.wavelet()
    d, uh = oracle.forward(grid, m0, src, rec, wav, return_history=True)
    _, lh = oracle.adjoint(grid, m0, src, rec, d - dobs, return_history=True)
    shape = tuple(wl.shape)
    u = uh[0]
    lam = np.concatenate([lh[0], np.zeros((1,) + shape)])
    a = u[1:]                                   # u^s, s = 1..nt-1
    b = lam[0:-2] - 2 * lam[1:-1] + lam[2:]     # w^s
    # exact imaging condition: grad applied to every pair of snapshots
    exact = -np.sum(_grad_dot(wl.h, a, b), axis=0)
    g_id, _ = oracle.gradient_probed(grid, m0, src, rec, wav, dobs, kind="identity", r=wl.nt, imaging=1)
    np.testing.assert_allclose(g_id, exact, rtol=0, atol=1e-11 * np.abs(exact).max())
    # random probes: grad of the probed fields == probed grad of the snapshots
    r, seed = 5, 23
    Z = oracle.probe_matrix("rademacher", r, seed, wl.nt, 0)[1:]          # rows s = 1..nt-1
    U = np.einsum("sj,s...->j...", Z, a)
    W = np.einsum("sj,s...->j...", Z, b)
    probed = -np.sum(_grad_dot(wl.h, U, W), axis=0) / r
    g_pr, _ = oracle.gradient_probed(grid, m0, src, rec, wav, dobs, kind="rademacher", r=r, seed=seed, imaging=1)
    np.testing.assert_allclose(g_pr, probed, rtol=0, atol=1e-11 * np.abs(probed).max())
    # and it differs from the pointwise imaging condition
    g_pt, _ = oracle.gradient_probed(grid, m0, src, rec, wav, dobs, kind="rademacher", r=r, seed=seed)
    assert np.abs(g_pt - g_pr).max() > 1e-3 * np.abs(g_pr).max()
