"""GPU: the probe-family study (studies.run) and the outer-product comparison
(studies.crosstalk) on a small 2D workload, against the FP64 oracle's exact
and probed gradients and its probing matrices."""
import math

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import Case, ensure_built

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="no GPU")]

import oracle  # noqa: E402
from paper_2104_00794_amd import studies  # noqa: E402
from paper_2104_00794_amd.inputs import small_2d  # noqa: E402

FAMILIES = ["rademacher", "gauss_b64", "range_finder", "fourier"]


def _wl():
    return small_2d(nz=36, nx=44, nt=160, nshots=2, nrec=9, seed=13)


def _oracle_probes(c, fam, r, seed, dobs):
    wl = c.wl
    if fam == "fourier":
        return studies.fourier_probes(wl.nt, wl.dt, wl.f_khz, r, wl.nshots).astype(np.float64), 1.0
    if fam == "range_finder":
        return oracle.range_finder_probes(dobs, r, seed), 1.0
    return np.stack([oracle.probe_matrix(fam, r, seed, wl.nt, s) for s in range(wl.nshots)]), 1.0 / r


def test_study_errors_match_the_oracle():
    ensure_built()
    wl = _wl()
    print(f"study: shape {wl.shape} nt {wl.nt} shots {wl.nshots}", flush=True)
    res = studies.run("small", [4, 8], FAMILIES, 1, [0, 1], wl=wl)
    c = Case(wl)
    dobs = c.dobs_oracle()
    g_ex, _ = oracle.gradient_full(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs)
    gn = np.linalg.norm(g_ex)
    assert len(res["rows"]) == len(FAMILIES) * 2 * 2
    for row in res["rows"]:
        fam, r, side = row["family"], row["r"], row["side"]
        seed = 1000 + r
        Z, scale = _oracle_probes(c, fam, r, seed, dobs)
        g_o, _ = oracle.gradient_probed(c.ogrid(), c.m0, c.src, c.rec, c.wav, dobs, kind="explicit", r=r,
                                        Z=Z, scale=scale, side=side)
        err = np.linalg.norm(g_o - g_ex) / gn
        print(fam, r, side, row["rel_err_mean"], err, flush=True)
        assert abs(row["rel_err_mean"] - err) <= 1e-3 * max(err, 1.0), (row, err)


def test_crosstalk_matches_the_oracle_probes():
    ensure_built()
    wl = _wl()
    rs = [4, 8, 16]
    res = studies.crosstalk("small", rs, FAMILIES, 2, wl=wl)
    c = Case(wl)
    dobs = c.dobs_oracle()
    V = studies.band_basis(wl.nt, wl.dt, wl.f_khz)
    rows = {(x["family"], x["r"]): x for x in res["rows"]}
    # the range finder stops at r = nrec (the rank of D D^T)
    assert len(rows) == len(FAMILIES) * len(rs) - sum(1 for r in rs if r > len(wl.rec))
    for (fam, r), row in rows.items():
        vals = []
        for s in range(row["seeds"]):
            Z, scale = _oracle_probes(c, fam, r, 1000 * (s + 1) + r, dobs)
            vals.append(studies.outer_distance(Z[0], scale, V))
        full, band = np.mean(vals, axis=0)
        tol = 1e-3 if fam == "range_finder" else 1e-5
        assert abs(row["full_mean"] - full) <= tol * full, (fam, r, row, full)
        assert abs(row["band_mean"] - band) <= tol * max(band, 1e-3), (fam, r, row, band)
        if fam in ("fourier", "range_finder"):
            # orthonormal columns: ||Q Q^T - I||_F^2 = n_t - r exactly
            assert abs(row["full_mean"] - math.sqrt((wl.nt - r) / wl.nt)) < 1e-4
