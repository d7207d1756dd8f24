#!/usr/bin/env python3
"""Throughput of the probed FWI gradient on one MI355X.

One step = one complete probed-gradient call (probe generation, forward
propagation with on-the-fly probing, residual and objective, adjoint
propagation with on-the-fly probing, imaging) over the whole shot batch, with
every input already resident in HBM.

Metric: GPts/s = shots * padded grid points * 2 (nt - 1) / wall time, the
grid-point updates of the forward and adjoint passes.  The JSON line also
carries the roofline of the dominant kernel (the leapfrog step), the p50/p99
latency of the gradient call, and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2104_00794_amd import profiling  # noqa: E402  (reads measured traffic records only)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1_layered_2d_16shots")
    ap.add_argument("--r", type=int, default=None, help="probes (default: the workload's)")
    ap.add_argument("--probe", default=None, help="rademacher | gauss_b64 | range_finder")
    ap.add_argument("--block", type=int, default=0, help="time steps per probe contraction (0 = default)")
    ap.add_argument("--keep-vbar", action="store_true", help="accumulate vbar instead of folding it")
    ap.add_argument("--full", action="store_true",
                    help="time the full-storage exact gradient (Eq. 3) instead of the probed one")
    ap.add_argument("--dtt-side", type=int, default=0, choices=[0, 1],
                    help="1: probe the second time difference of u and lambda itself (Algorithm 1 as printed)")
    ap.add_argument("--imaging", type=int, default=0, choices=[0, 1],
                    help="1: image the probed fields through their spatial gradients (Eq. 5; keeps vbar)")
    ap.add_argument("--overlap", action="store_true",
                    help="run the probe contractions on the auxiliary stream, overlapping the next time block")
    ap.add_argument("--matrix-cores", type=int, default=None, choices=[0, 1, 2],
                    help="probe contractions on the matrix cores: 0 never, 1 for r >= 32 (library default), 2 always")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter calibration)")
    ap.add_argument("--nt", type=int, default=None, help="override the record length (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-nt", type=int, default=0, help="time steps of the CPU-oracle sample (0 = full record)")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="serving mix instead: continuous batching vs one-at-a-time on one Poisson trace")
    ap.add_argument("--requests", type=int, default=60, help="requests in the serving trace")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="HBM budget of the server")
    ap.add_argument("--chunk-steps", type=int, default=64, help="time steps a served job advances per turn")
    ap.add_argument("--max-active", type=int, default=3,
                    help="jobs the server keeps on the GPU at once (default: one fewer than the hardware queues)")
    ap.add_argument("--inflight", type=int, default=2, help="chunks each served job keeps queued")
    ap.add_argument("--large-points", type=float, default=3e6,
                    help="padded points over a job's shots from which it counts as large")
    ap.add_argument("--max-large", type=int, default=2, help="large jobs the server runs at once")
    ap.add_argument("--c3-steps", type=int, default=3,
                    help="timed gradient calls of the 3D workload for the c3 sub-record (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="requests of the serving sub-record (0: skip)")
    ap.add_argument("--fused-3d", type=int, default=None, choices=[0, 1],
                    help="two leapfrog steps per 3D launch (library option; default: the library's)")
    ap.add_argument("--steps-2d", type=int, default=None, choices=[2, 3],
                    help="most leapfrog steps per 2D launch (default: the library's, 3)")
    return ap.parse_args()


def stencil_bytes(S: int) -> float:
    """Algorithmic HBM bytes of one leapfrog step per shot and padded point: read
    u^k and u^{k-1}, write u^{k+1}, and beta read once for the S batched shots."""
    return 12.0 + 4.0 / S


def path_bytes(S: int, phi: float) -> float:
    """Algorithmic bytes per shot-point-step of the whole probed path: the
    stencil, plus one re-read of each probed sample by the time-blocked
    contraction (phi = physical / padded points)."""
    return stencil_bytes(S) + 4.0 * phi


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs the whole gradient of a shot batch on a single "
              "MI355X and has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_00794_amd import build as tbuild
    if not os.path.exists(tbuild.LIB_PATH):
        tbuild.build(force=True)
    from paper_2104_00794_amd import tpx
    from paper_2104_00794_amd.inputs import workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32 read and 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}), flush=True)
        return
    tpx.set_option(tpx.OPT_OVERLAP_CONTRACTIONS, 1 if args.overlap else 0)
    if args.matrix_cores is not None:
        tpx.set_option(tpx.OPT_MATRIX_CORES, args.matrix_cores)
    if args.fused_3d is not None:
        tpx.set_option(tpx.OPT_FUSED_STEPS_3D, args.fused_3d)
    if args.steps_2d is not None:
        tpx.set_option(tpx.OPT_STEPS_2D, args.steps_2d)
    if args.serving:
        print(json.dumps(serving(args, dev)), flush=True)
        return

    wl = workload(args.workload)
    if args.nt:
        wl = wl.with_(nt=args.nt)
    rec = gradient_record(args, wl, args.steps, args.warmup, dev, profile=not args.no_profile_pass)
    progress("headline workload %s done: %.1f GPts/s" % (wl.name, rec["value"]))

    # ---- reference rate: a plain device copy of 1 GiB (after the timed region) ------------
    copy_gbps = None if args.no_profile_pass else copy_bandwidth(dev)

    # ---- the 3D workload whose full-storage gradient cannot fit on the GPU ------------------
    c3 = None
    if args.c3_steps > 0 and args.workload != "c3_layered_3d" and not args.full:
        wl3 = workload("c3_layered_3d")
        torch.cuda.empty_cache()
        r3 = gradient_record(args, wl3, args.c3_steps, 1, dev, profile=not args.no_profile_pass, default_probe=True)
        c3 = {k: r3[k] for k in ("value", "unit", "value_physical_points", "ms_per_step", "steps", "latency_ms",
                                  "hbm_roofline_pct", "b_alg_bytes_per_point_step", "roofline", "memory",
                                  "workspace_GB", "kernels", "config", "J")}
        torch.cuda.empty_cache()
        progress("c3 done: %.1f GPts/s" % c3["value"])

    # ---- serving mix: continuous batching against the plain path ---------------------------
    srv = None
    if args.serving_requests > 0 and not args.full:
        sargs = argparse.Namespace(**vars(args))
        sargs.requests = args.serving_requests
        sargs.saturation = False
        srv = serving(sargs, dev)
        progress("serving done")

    # ---- CPU baseline: the FP64 oracle on a bounded sample ---------------------------------
    cpu = None
    if not args.no_cpu_baseline and not args.full:
        # about 10-30 s of oracle work in all: the full record of a few 2D
        # shots, or a short window of the 3D record, timed three times
        cpu = cpu_baseline(wl, rec["config"]["r"], rec["config"]["probe"],
                           args.cpu_nt or (wl.nt if wl.ndim == 2 else 8),
                           min(2, wl.nshots) if wl.ndim == 2 else 1, reps=3)

    out = {
        "metric": "GPts/s fwd+adj with r-probe accumulation (%HBM roofline); gradient p50/p99 latency",
        "value": rec["value"],
        "unit": "GPts/s",
        "value_physical_points": rec["value_physical_points"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": rec["config"],
        "gradient": rec["gradient"],
        "workspace_GB": rec["workspace_GB"],
        "memory": rec["memory"],
        "host_enqueue_ms": rec["host_enqueue_ms"],
        "latency_ms": rec["latency_ms"],
        "hbm_roofline_pct": rec["hbm_roofline_pct"],
        "b_alg_bytes_per_point_step": rec["b_alg_bytes_per_point_step"],
        "hbm_roofline_pct_stencil_only": rec["hbm_roofline_pct_stencil_only"],
        "roofline": rec["roofline"],
        "roofline_fused_launch": rec["roofline_fused_launch"],
        "copy_GBps": copy_gbps,
        "kernels": rec["kernels"],
        "kernel_timing": "HIP events on the launch stream around each run of consecutive launches of one "
                         "kernel kind, in one profiled call after the timed region",
        "c3": c3,
        "serving": srv,
        "cpu_baseline": cpu,
        "J": rec["J"],
    }
    print(json.dumps(out), flush=True)


def progress(msg: str) -> None:
    print("bench: " + msg, file=sys.stderr, flush=True)


def gradient_record(args, wl, steps, warmup, dev, profile=True, default_probe=False):
    """Time `steps` complete gradient calls of workload `wl` (inputs resident in
    HBM), then one profiled call for the per-kernel durations."""
    import torch
    from paper_2104_00794_amd import tpx
    r = wl.r if default_probe else (args.r or wl.r)
    kind = wl.probe if default_probe else (args.probe or wl.probe)
    keep_vbar = False if default_probe else bool(args.keep_vbar or args.imaging)
    dtt_side = 0 if default_probe else args.dtt_side
    imaging = 0 if default_probe else args.imaging
    block = 0 if default_probe else args.block
    full = False if default_probe else args.full
    mt, m0 = wl.models()
    grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax,
                    damp_R=wl.damp_R)
    wav = torch.tensor(wl.wavelet(), dtype=torch.float32, device=dev)
    geom = tpx.Geometry(wl.src_pos(), wl.rec_pos(), wav)
    m_true = torch.tensor(mt, dtype=torch.float32, device=dev)
    m_0 = torch.tensor(m0, dtype=torch.float32, device=dev)
    del mt, m0
    probe = tpx.Probe(kind=kind, r=r, seed=wl.probe_seed, block=block, keep_vbar=keep_vbar,
                      dtt_side=dtt_side, imaging=imaging)

    d_obs = tpx.forward(grid, geom, m_true)           # synthetic observed data (untimed input)
    del m_true
    ws = tpx.alloc_workspace(tpx.CALL_GRADIENT_FULL if full else tpx.CALL_GRADIENT_PROBED, grid, geom,
                             None if full else probe, dev)
    g = torch.empty(tuple(wl.shape), dtype=torch.float32, device=dev)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        if full:   # the exact gradient from the stored history (Eq. 3), for comparison
            g_f, J_f = tpx.gradient_full(grid, geom, m_0, d_obs, ws=ws, stream=stream)
            g.copy_(g_f)
            J.copy_(J_f)
        else:
            tpx.gradient_probed(grid, geom, probe, m_0, d_obs, ws=ws, g_out=g, J_out=J, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tpx.check_workspace(ws)

    # ---- timed region: `steps` complete gradient calls ------------------------------------
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    # host time to enqueue one call (the call returns once its work is queued)
    torch.cuda.synchronize()
    th = time.perf_counter()
    step()
    host_enqueue_ms = (time.perf_counter() - th) * 1e3
    torch.cuda.synchronize()

    S, npad, nphys, nt = wl.nshots, wl.n_pad, wl.n_phys, wl.nt
    updates = S * npad * 2 * (nt - 1)
    gpts = updates / (ms_per_step * 1e-3) / 1e9
    phi = nphys / npad
    b_alg = path_bytes(S, phi)

    # ---- per-kernel durations (HIP events on the launch stream) ----------------------------
    kernels = {}
    roofline = fused = None
    if profile:
        tpx.profile_enable(True)
        step()
        torch.cuda.synchronize()
        for name, kid in (("step3", tpx.KERNEL_STEP3), ("step2", tpx.KERNEL_STEP2), ("step", tpx.KERNEL_STEP),
                          ("accum_fwd", tpx.KERNEL_ACCUM_FWD), ("accum_adj", tpx.KERNEL_ACCUM_ADJ),
                          ("accum_full", tpx.KERNEL_ACCUM_FULL)):
            tot, n = tpx.profile_read(kid)
            kernels[name] = {"total_ms": round(tot, 4), "launches": n,
                             "avg_us": round(1e3 * tot / n, 3) if n else None}
        tpx.profile_enable(False)
        # dominant kernel: the step kernel kind with the largest total time
        dom = max(("step3", "step2", "step"), key=lambda n: kernels[n]["total_ms"])
        st = kernels[dom]
        nstep = {"step3": 3, "step2": 2, "step": 1}[dom]
        R = wl.order // 2
        if wl.ndim == 2:
            kname = "k_step2d3<R=%d>" % R if nstep == 3 else "k_step2d<R=%d,NSTEP=%d>" % (R, nstep)
            tag = {3: "k_step2d_x3", 2: "k_step2d_x2", 1: "k_step2d"}[nstep]
        else:
            kname, tag = ("k_step3d2<R=%d>" % R, "k_step3d2") if nstep == 2 else ("k_step3d<R=%d>" % R, "k_step3d")
        if st["launches"]:
            # the paper's leapfrog traffic per shot-point-step, times the steps one launch advances
            bytes_per_launch = nstep * S * npad * stencil_bytes(S)
            achieved = bytes_per_launch / (st["avg_us"] * 1e-6) / 1e9
            traffic = profiling.read_traffic(wl.name, tag)   # None unless measured with this kernel source
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                        "steps_per_launch": nstep, "bytes_per_launch": bytes_per_launch,
                        "bytes_per_shot_point_step": round(stencil_bytes(S), 4), "avg_launch_us": st["avg_us"]}
            # what a launch of nstep fused steps must move at least: u^{k-1}, u^k and beta once,
            # nstep new levels written
            fb = S * npad * (8.0 + 4.0 * nstep) + npad * 4.0
            fa = fb / (st["avg_us"] * 1e-6) / 1e9
            fused = {"bytes_per_launch": fb, "achieved": round(fa, 1), "frac": round(fa / HBM_PEAK_GBS, 4)}

    # ---- memory: probed workspace against the stored forward history -----------------------
    hist = S * nphys * nt * 4.0                       # the history of Eq. 3 (N x n_t values per shot)
    full_ws = tpx.workspace_bytes(tpx.CALL_GRADIENT_FULL, grid, geom, None)
    memory = {"workspace_GB": round(ws.numel() / 1e9, 3),
              "history_GB": round(hist / 1e9, 3),
              "full_storage_workspace_GB": round(full_ws / 1e9, 3),
              "accumulators_GB": round(S * r * nphys * 4.0 / 1e9, 3),
              "reduction_vs_history": round(hist / ws.numel(), 2),
              "paper_reduction_nt_over_2r": round(nt / (2.0 * r), 2)}

    return {
        "value": round(gpts, 3), "unit": "GPts/s", "value_physical_points": round(gpts * phi, 3),
        "steps": steps, "ms_per_step": round(ms_per_step, 3),
        "config": {"workload": wl.name, "grid": "x".join(str(s) for s in wl.shape[::-1]), "h_m": wl.h,
                   "space_order": wl.order, "shots": S, "nt": nt, "nbl": wl.nbl, "r": r, "probe": kind,
                   "block": block or "default", "keep_vbar": keep_vbar, "dtt_side": dtt_side, "imaging": imaging,
                   "overlap_contractions": bool(tpx.get_option(tpx.OPT_OVERLAP_CONTRACTIONS)),
                   "fused_steps_3d": bool(tpx.get_option(tpx.OPT_FUSED_STEPS_3D)),
                   "max_steps_per_launch_2d": tpx.get_option(tpx.OPT_STEPS_2D),
                   "matrix_core_contractions": matrix_core_use(kind, r, keep_vbar),
                   "padded_points_per_shot": npad, "parallelism": "single-gpu"},
        "gradient": "full-storage (Eq. 3)" if full else "probed (Eq. 4)",
        "workspace_GB": round(ws.numel() / 1e9, 3),
        "memory": memory,
        "host_enqueue_ms": round(host_enqueue_ms, 2),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3)},
        "hbm_roofline_pct": round(100.0 * gpts * b_alg / HBM_PEAK_GBS, 2),
        "b_alg_bytes_per_point_step": round(b_alg, 3),
        # the stencil's bytes alone (12 + 4/S), without the probe re-read
        "hbm_roofline_pct_stencil_only": round(100.0 * gpts * stencil_bytes(S) / HBM_PEAK_GBS, 2),
        "roofline": roofline,
        "roofline_fused_launch": fused,
        "kernels": kernels,
        "J": float(J.item()),
    }


def serving(args, dev):
    """Serving mix: p50/p99 latency and aggregate GPts/s, continuous batching vs
    the plain one-at-a-time path on the same Poisson arrival trace (and, with
    `args.saturation`, with every request queued at once)."""
    import torch
    from paper_2104_00794_amd import serve, tpx
    from paper_2104_00794_amd.inputs import serving_workload
    reqs = []
    for i in range(args.requests):
        wl = serving_workload(i, 41)
        mt, m0 = wl.models()
        grid = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
        geom = tpx.Geometry(wl.src_pos(), wl.rec_pos(), torch.tensor(wl.wavelet(), dtype=torch.float32, device=dev))
        d_obs = tpx.forward(grid, geom, torch.tensor(mt, dtype=torch.float32, device=dev))
        # a 256-level ring per request keeps many jobs inside the server's budget
        reqs.append(serve.Request(i, grid, geom, tpx.Probe(r=wl.r, seed=wl.probe_seed, block=256),
                                  torch.tensor(m0, dtype=torch.float32, device=dev), d_obs))
    torch.cuda.synchronize()
    print("serving: %d requests prepared" % len(reqs), file=sys.stderr, flush=True)
    # service time of the plain path (also the warm-up), then the arrival rate
    svc = serve.run_sequential(reqs)
    mean_service = float(np.mean([r.finished - r.admitted for r in svc.values()]))
    rate = 0.8 / mean_service
    arr = serve.poisson_arrivals(len(reqs), rate, 41)
    for q, a in zip(reqs, arr):
        q.arrival = float(a)
    seq = serve.run_sequential(reqs)
    print("serving: plain path on the Poisson trace done", file=sys.stderr, flush=True)
    srv = serve.Server(hbm_budget_bytes=args.budget_gb * 1e9, chunk_steps=args.chunk_steps,
                       max_active=args.max_active, nstreams=8, inflight=args.inflight,
                       large_points=args.large_points, max_large=args.max_large)
    bat = srv.run(reqs)
    same = all(torch.equal(seq[q.rid].g, bat[q.rid].g) for q in reqs if bat[q.rid].status == "ok")
    a, b = serve.summarize(seq, reqs), serve.summarize(bat, reqs)
    print("serving: server on the Poisson trace done", file=sys.stderr, flush=True)
    saturated = None
    if getattr(args, "saturation", True):
        # saturation: every request queued at once, so the makespan measures how
        # much work the GPU absorbs when jobs overlap (small grids alone leave most
        # of the 256 CUs idle)
        for q in reqs:
            q.arrival = 0.0
        sat_seq = serve.summarize(serve.run_sequential(reqs), reqs)
        print("serving: plain path at saturation done", file=sys.stderr, flush=True)
        srv2 = serve.Server(hbm_budget_bytes=args.budget_gb * 1e9, chunk_steps=args.chunk_steps,
                            max_active=args.max_active, nstreams=8, inflight=args.inflight,
                            large_points=args.large_points, max_large=args.max_large)
        sat_bat = serve.summarize(srv2.run(reqs), reqs)
        saturated = {"batched": sat_bat, "sequential": sat_seq,
                     "throughput_ratio": round(sat_bat["gpts_per_s"] / sat_seq["gpts_per_s"], 3)}
    out = {
        "metric": "serving: gradient p50/p99 latency and aggregate GPts/s, continuous batching vs one-at-a-time",
        "value": b["gpts_per_s"], "unit": "GPts/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic", "vs_baseline": None,
        "config": {"workload": "serving mix: 2D 201x201..1001x401 (1-32 shots), 3D 201^3 (1 shot), "
                               "r in {8,32,64}, order 8", "requests": len(reqs),
                   "arrival": "Poisson, %.2f req/s = 0.8 x sequential service rate" % rate,
                   "hbm_budget_gb": args.budget_gb, "chunk_steps": args.chunk_steps,
                   "max_active": args.max_active, "inflight": args.inflight,
                   "large_points": args.large_points, "max_large": args.max_large},
        "batched": b, "sequential": a, "mean_service_ms": round(1e3 * mean_service, 2),
        "p99_ratio_sequential_over_batched": round(a["p99_ms"] / b["p99_ms"], 3),
        "p50_ratio_sequential_over_batched": round(a["p50_ms"] / b["p50_ms"], 3),
        "saturated": saturated,
        "peak_active_jobs": srv.peak_active, "peak_workspace_gb": round(srv.peak_bytes / 1e9, 2),
        "results_identical": bool(same),
    }
    del reqs, seq, bat
    return out


def cpu_baseline(wl, r, kind, nt_sample, shots, reps=3):
    """FP64 oracle on the first `shots` shots of the workload, first nt_sample
    time steps; the median of `reps` timed runs."""
    import oracle
    oracle.build(force=False)
    sample = wl.with_(nt=nt_sample, src=wl.src[:shots])
    mt, m0 = sample.models()
    og = oracle.Grid(sample.shape, h=sample.h, dt=sample.dt, nt=sample.nt, order=sample.order, nbl=sample.nbl,
                     damp_vmax=sample.vmax, damp_R=sample.damp_R)
    # the sample's observed traces, modelled by the oracle itself (untimed)
    dobs = oracle.forward(og, mt, sample.src_pos(), sample.rec_pos(), sample.wavelet())
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        if kind == "range_finder":
            Q = oracle.range_finder_probes(dobs, r, sample.probe_seed)
            oracle.gradient_probed(og, m0, sample.src_pos(), sample.rec_pos(), sample.wavelet(), dobs,
                                   kind="explicit", r=r, Z=Q, scale=1.0)
        else:
            oracle.gradient_probed(og, m0, sample.src_pos(), sample.rec_pos(), sample.wavelet(), dobs, kind=kind,
                                   r=r, seed=sample.probe_seed)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    upd = sample.nshots * sample.n_pad * 2 * (sample.nt - 1)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(upd / dt / 1e9, 5), "unit": "GPts/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "runs": reps, "statistic": "median",
            "seconds": [round(t, 2) for t in times],
            "sample": "%d of %d shots, first %d of %d time steps, r=%d %s, same grid; FP64 C oracle with OpenMP"
                      % (sample.nshots, wl.nshots, sample.nt, wl.nt, r, kind)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(dev, n: int = 1 << 28, reps: int = 5) -> float:
    """Read + write bytes per second of a plain 1 GiB device copy (median of `reps`), GB/s:
    the rate a pure streaming kernel reaches on this HBM."""
    import torch
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    return round(2.0 * 4 * n / float(np.median(times)) / 1e9, 1)


def matrix_core_use(kind: str, r: int, keep_vbar: bool) -> str:
    """Which contractions run on the matrix cores under the library option."""
    from paper_2104_00794_amd import tpx
    opt = tpx.get_option(tpx.OPT_MATRIX_CORES)
    if r % 16 != 0 or opt == 0:
        return "none"
    accum = opt == 2 or r >= 64
    fold = not keep_vbar and (opt == 2 or r >= 32)
    parts = [p for p, on in (("ubar", accum), ("vbar", accum and keep_vbar), ("fold", fold)) if on]
    return "+".join(parts) or "none"


if __name__ == "__main__":
    main()
