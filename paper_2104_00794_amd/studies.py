"""Accuracy of the probed gradient against the exact one, by probe family.

For one workload: the exact gradient (Eq. 3, full history) and probed
gradients (Eq. 4, Algorithm 1) for several probing families and numbers of
probes r, on both sides of the second time difference.  Families:

* ``rademacher``, ``gauss_b64``: i.i.d. probes (Randomized trace estimation);
* ``range_finder``: Q = qr(D_obs D_obs^T Z) per shot (Choice of the probing
  matrix Q, Eq. 6);
* ``fourier``: a restricted Fourier basis, r/2 frequencies spread uniformly
  over the source band [f/4, 5f/2] (cosine and sine columns, orthonormalised),
  the paper's comparison family in the same section.

Reports the relative L2 error ||g~ - g|| / ||g|| over the physical grid and its
spread over seeds.  Everything runs on the GPU through the library.

``crosstalk`` measures Fig. 1's comparison of the outer products Z Z^T
(i.i.d.), F F^T (restricted Fourier) and Q Q^T (range finder), each scaled as
the gradient uses it (c Z Z^T, c = 1/r for i.i.d. probes, 1 for orthonormal
ones), by its distance from the identity: over the whole time axis,
||c Z Z^T - I||_F / sqrt(n_t), and inside the source band, where the wavefields
and their time correlations live, ||V^T (c Z Z^T - I) V||_F / sqrt(n_B) with V
an orthonormal basis of the band (n_B columns).  The i.i.d. and range-finder
probes are the ones the GPU generates.

    python -m paper_2104_00794_amd.studies --workload c1_layered_2d_16shots
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import tpx
from .inputs import workload


def fourier_probes(nt: int, dt: float, f_khz: float, r: int, nshots: int) -> np.ndarray:
    """Orthonormal restricted Fourier basis [S][nt][r] (the same for every shot)."""
    t = np.arange(nt) * dt
    freqs = np.linspace(0.25 * f_khz, 2.5 * f_khz, (r + 1) // 2)
    cols = []
    for f in freqs:
        cols.append(np.cos(2 * math.pi * f * t))
        cols.append(np.sin(2 * math.pi * f * t))
    F = np.stack(cols[:r], axis=1)
    Q = np.linalg.qr(F, mode="reduced")[0]
    return np.broadcast_to(Q, (nshots, nt, r)).astype(np.float32).copy()


def band_basis(nt: int, dt: float, f_khz: float) -> np.ndarray:
    """Orthonormal basis [nt][n_B] of the real signals of the source band
    [f/4, 5f/2]: the cosines and sines of the record's DFT frequencies there."""
    t = np.arange(nt) * dt
    T = nt * dt
    ks = [k for k in range(1, nt // 2) if 0.25 * f_khz <= k / T <= 2.5 * f_khz]
    cols = [g(2 * math.pi * (k / T) * t) for k in ks for g in (np.cos, np.sin)]
    return np.linalg.qr(np.stack(cols, axis=1), mode="reduced")[0]


def outer_distance(Z: np.ndarray, c: float, V: np.ndarray):
    """(||c Z Z^T - I||_F / sqrt(n_t), ||V^T (c Z Z^T - I) V||_F / sqrt(n_B))
    for Z [nt][r], evaluated through r x r and n_B x r products."""
    Z = np.asarray(Z, dtype=np.float64)
    nt, nb = Z.shape[0], V.shape[1]
    G = Z.T @ Z
    full2 = c * c * float(np.sum(G * G)) - 2.0 * c * float(np.trace(G)) + nt
    W = V.T @ Z
    Gb = W.T @ W
    band2 = c * c * float(np.sum(Gb * Gb)) - 2.0 * c * float(np.trace(Gb)) + nb
    return math.sqrt(max(full2, 0.0) / nt), math.sqrt(max(band2, 0.0) / nb)


def crosstalk(name, rs, families, seeds: int, device="cuda", wl=None):
    """Fig. 1's outer-product comparison, shot 0's probes, as r grows."""
    import torch
    wl = wl or workload(name)
    V = band_basis(wl.nt, wl.dt, wl.f_khz)
    d_obs = geom = grid = None
    if "range_finder" in families:
        mt, _ = wl.models()
        grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
        geom = tpx.Geometry(wl.src_pos(), wl.rec_pos(),
                            torch.tensor(wl.wavelet(), dtype=torch.float32, device=device))
        d_obs = tpx.forward(grid, geom, torch.tensor(mt, dtype=torch.float32, device=device))
    rows = []
    for fam in families:
        for r in rs:
            if fam == "range_finder" and r > min(64, geom.nrec, wl.nt):
                continue
            vals = []
            for s in range(seeds if fam != "fourier" else 1):
                seed = 1000 * (s + 1) + r
                if fam == "fourier":
                    Z, c = fourier_probes(wl.nt, wl.dt, wl.f_khz, r, 1)[0], 1.0
                elif fam == "range_finder":
                    Q = tpx.range_finder_probes(grid, geom, tpx.Probe(kind="range_finder", r=r, seed=seed), d_obs)
                    Z, c = Q[0].double().cpu().numpy(), 1.0
                else:
                    Z = tpx.probe_matrix(tpx.Probe(kind=fam, r=r, seed=seed), wl.nt, 0, device=device)
                    Z, c = Z.double().cpu().numpy(), 1.0 / r
                vals.append(outer_distance(Z, c, V))
            v = np.array(vals)
            rows.append({"family": fam, "r": r, "seeds": len(vals), "n_t": wl.nt, "n_band": V.shape[1],
                         "full_mean": float(v[:, 0].mean()), "band_mean": float(v[:, 1].mean())})
            print(json.dumps(rows[-1]), flush=True)
    return {"workload": wl.name, "rows": rows}


def run(name: str, rs, families, seeds: int, sides, device="cuda", wl=None):
    import torch
    wl = wl or workload(name)
    mt, m0 = wl.models()
    grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
    wav = torch.tensor(wl.wavelet(), dtype=torch.float32, device=device)
    geom = tpx.Geometry(wl.src_pos(), wl.rec_pos(), wav)
    m_true = torch.tensor(mt, dtype=torch.float32, device=device)
    m_0 = torch.tensor(m0, dtype=torch.float32, device=device)
    d_obs = tpx.forward(grid, geom, m_true)
    g_exact, _ = tpx.gradient_full(grid, geom, m_0, d_obs)
    gn = torch.linalg.vector_norm(g_exact.double()).item()
    rows = []
    for fam in families:
        for r in rs:
            if fam == "range_finder" and r > min(64, geom.nrec, wl.nt):
                continue
            for side in sides:
                errs = []
                for s in range(seeds if fam != "fourier" else 1):
                    seed = 1000 * (s + 1) + r
                    if fam == "fourier":
                        Z = torch.tensor(fourier_probes(wl.nt, wl.dt, wl.f_khz, r, wl.nshots), device=device)
                        probe = tpx.Probe(kind="explicit", r=r, Z=Z, scale=1.0, dtt_side=side)
                    else:
                        probe = tpx.Probe(kind=fam, r=r, seed=seed, dtt_side=side)
                    g, _ = tpx.gradient_probed(grid, geom, probe, m_0, d_obs)
                    errs.append(torch.linalg.vector_norm((g - g_exact).double()).item() / gn)
                rows.append({"family": fam, "r": r, "side": side, "seeds": len(errs),
                             "rel_err_mean": float(np.mean(errs)), "rel_err_min": float(np.min(errs)),
                             "rel_err_max": float(np.max(errs))})
                print(json.dumps(rows[-1]), flush=True)
    return {"workload": name, "nt": wl.nt, "shots": wl.nshots, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="c1_layered_2d_16shots")
    ap.add_argument("--r", type=int, nargs="+", default=[4, 8, 16, 32, 64])
    ap.add_argument("--families", nargs="+", default=["rademacher", "gauss_b64", "range_finder", "fourier"])
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--sides", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--out", default=None, help="write the result as JSON")
    ap.add_argument("--crosstalk", action="store_true", help="Fig. 1's outer-product comparison instead")
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    if a.crosstalk:
        res = crosstalk(a.workload, a.r, a.families, a.seeds)
    else:
        res = run(a.workload, a.r, a.families, a.seeds, a.sides)
    res["seconds"] = round(time.perf_counter() - t0, 1)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({"seconds": res["seconds"]}))


if __name__ == "__main__":
    main()
