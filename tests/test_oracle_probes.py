"""Pins of the oracle's probe generator (Philox4x64-10 counter hash).

* known-answer vectors published with the generator (tests/golden);
* NumPy's independent Philox implementation reproduces every entry;
* Rademacher entries are +-1; Gauss-B64 entries are k/4 with the moments of a
  centred Binomial(64, 1/2) / 4 (mean 0, variance 1, kurtosis 3 - 2/64);
* E ||Z Z^T / r - I||_F^2 matches its closed form (the cross-talk of the
  Choice-of-the-probing-matrix section).
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox4x64_10(ctr, key) == out


def _numpy_block(seed, t, j, shot):
    # NumPy's Philox increments its 256-bit counter before producing a block,
    # so counter (t, j, shot, 0) yields the block at (t + 1, j, shot, 0).
    g = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                         counter=np.array([t, j, shot, 0], dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("kind", ["rademacher", "gauss_b64"])
def test_probe_matrix_matches_numpy_philox(kind):
    nt, r = 23, 7
    for seed, shot in ((0, 0), (12, 3), (2**63 + 5, 15)):
        Z = oracle.probe_matrix(kind, r, seed, nt, shot)
        for t in range(nt):
            for j in range(r):
                w0 = int(_numpy_block(seed, t, j, shot)[0])
                if kind == "rademacher":
                    z = 1.0 - 2.0 * (w0 >> 63)
                else:
                    z = (bin(w0).count("1") - 32) / 4.0
                assert Z[t, j] == z


def test_rademacher_entries():
    Z = oracle.probe_matrix("rademacher", 64, 7, 500, 2)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert abs(Z.mean()) < 5 / np.sqrt(Z.size)


def test_gauss_b64_moments():
    Z = np.concatenate([oracle.probe_matrix("gauss_b64", 100, 3, 1000, s).ravel() for s in range(2)])
    k = Z * 4
    assert np.all(k == np.round(k)) and np.abs(k).max() <= 32
    n = Z.size
    assert abs(Z.mean()) < 5 / np.sqrt(n)
    assert abs(Z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    kurt = np.mean(Z ** 4) / np.mean(Z ** 2) ** 2
    assert abs(kurt - (3.0 - 2.0 / 64.0)) < 0.03


def test_identity_probe():
    Z = oracle.probe_matrix("identity", 9, 0, 9, 0)
    np.testing.assert_array_equal(Z, np.eye(9))
    with pytest.raises(oracle.OracleError):
        oracle.probe_matrix("identity", 8, 0, 9, 0)


@pytest.mark.parametrize("kind,kappa", [("rademacher", 1.0), ("gauss_b64", 3.0 - 2.0 / 64.0)])
def test_crosstalk_closed_form(kind, kappa):
    nt, r, nseed = 40, 8, 200
    vals = []
    for s in range(nseed):
        Z = oracle.probe_matrix(kind, r, 50 + s, nt, 0)
        E = Z @ Z.T / r - np.eye(nt)
        vals.append(np.sum(E ** 2))
    pred = nt * (nt - 1) / r + nt * (kappa - 1.0) / r
    assert abs(np.mean(vals) / pred - 1.0) < 0.05, (np.mean(vals), pred)


def test_shots_and_seeds_give_independent_streams():
    a = oracle.probe_matrix("rademacher", 16, 1, 64, 0)
    b = oracle.probe_matrix("rademacher", 16, 1, 64, 1)
    c = oracle.probe_matrix("rademacher", 16, 2, 64, 0)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert abs(np.mean(a * b)) < 0.15 and abs(np.mean(a * c)) < 0.15


# --------------------------------------------------------------------------- #
# probes from the range of the data covariance (Eq. 6)
# --------------------------------------------------------------------------- #

def _numpy_rademacher(seed, nt, r, shot):
    Z = np.empty((nt, r))
    for t in range(nt):
        for j in range(r):
            Z[t, j] = 1.0 - 2.0 * (int(_numpy_block(seed, t, j, shot)[0]) >> 63)
    return Z


def test_range_finder_probes_are_orthonormal_and_span_AZ():
    rng = np.random.default_rng(3)
    S, nt, nrec, r, seed = 2, 90, 25, 7, 41
    D = rng.standard_normal((S, nt, nrec)).astype(np.float32)
    Q = oracle.range_finder_probes(D, r, seed)
    assert Q.shape == (S, nt, r)
    for s in range(S):
        assert np.abs(Q[s].T @ Q[s] - np.eye(r)).max() <= 1e-12
        # A formed explicitly, Z from NumPy's own Philox stream of this shot
        A = D[s].astype(np.float64) @ D[s].T.astype(np.float64)
        Y = A @ _numpy_rademacher(seed, nt, r, s)
        resid = Y - Q[s] @ (Q[s].T @ Y)
        assert np.linalg.norm(resid) <= 1e-11 * np.linalg.norm(Y)
    # another shot's Z spans a different space
    Y0 = D[0].astype(np.float64) @ (D[0].T.astype(np.float64) @ _numpy_rademacher(seed, nt, r, 1))
    assert np.linalg.norm(Y0 - Q[0] @ (Q[0].T @ Y0)) > 1e-3 * np.linalg.norm(Y0)


def test_range_finder_recovers_the_trace_of_a_low_rank_covariance():
    # rank(D D^T) = k <= r: A Z spans the whole range of A, so the probed trace
    # tr(Q^T A Q) (c = 1) equals tr(A) = ||D||_F^2 exactly up to rounding,
    # while r Rademacher probes (c = 1/r) do not
    rng = np.random.default_rng(8)
    nt, nrec, k, r = 120, 40, 3, 5
    D = (rng.standard_normal((nt, k)) @ rng.standard_normal((k, nrec)))[None]
    Q = oracle.range_finder_probes(D, r, seed=9)[0]
    A = D[0] @ D[0].T
    tr = np.sum(D[0] ** 2)
    assert abs(np.trace(Q.T @ A @ Q) - tr) <= 1e-10 * tr
    Z = oracle.probe_matrix("rademacher", r, 9, nt, 0)
    assert abs(np.trace(Z.T @ A @ Z) / r - tr) > 1e-3 * tr
