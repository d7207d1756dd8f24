"""Continuous-batching server for probed-gradient requests on one GPU.

Requests (a grid, its acquisition, probes, the current model and the observed
data, all resident on the device) arrive over time.  The server admits a
request as soon as a slot is free and its workspace fits the HBM budget
(``tpx_workspace_bytes`` gives the exact size), then advances every admitted
job by a chunk of time steps at a time on its own HIP stream, so the work of
several jobs overlaps on the device; requests that arrive while others run
join at the next chunk boundary.  A job's results do not depend on its
neighbours (separate workspaces, deterministic kernels).

A request may be withdrawn (``Request.cancel_at``): waiting, it leaves the
queue; running, it stops advancing and its workspace is freed as soon as the
chunks already queued on its stream have run, without touching the others.

Job workspaces come from one device arena allocated when ``run`` starts
(``Arena``: first fit, coalescing frees), so no device allocation happens while
jobs run: a device allocation can wait for the GPU to drain, and measured
stalls of up to 0.75 s in the host loop otherwise.

``run_sequential`` is the plain path: one ``tpx_gradient_probed`` call at a
time in arrival order, on the same arrival trace, with one workspace of the
largest size allocated beforehand and reused.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import tpx


def admission_plan(waiting: Sequence, slots: int, free_bytes: float, budget: float, nlarge: int, max_large: int,
                   need: Callable, large: Callable):
    """The waiting requests to admit now and those to reject, scanned in arrival
    order: a request needing more than the whole budget is rejected; a large one
    is passed over while `max_large` large jobs run (smaller ones behind it may
    go first); the first request that does not fit the free bytes ends the
    scan, so memory is granted in arrival order.  At most `slots` are admitted.
    need(req) gives a request's device bytes, large(req) whether it is large."""
    admit, reject = [], []
    for req in waiting:
        if len(admit) >= slots:
            break
        n = need(req)
        if n > budget:
            reject.append(req)
            continue
        lg = bool(large(req))
        if lg and nlarge >= max_large:
            continue
        if n > free_bytes:
            break
        admit.append(req)
        free_bytes -= n
        nlarge += lg
    return admit, reject


class Arena:
    """One device allocation carved into workspaces: first fit over a free list
    kept in address order, adjacent free blocks merged on release.  Offsets
    and sizes are multiples of ALIGN bytes."""
    ALIGN = 4096

    def __init__(self, nbytes: int, device=None, buf=None):
        self.size = -(-int(nbytes) // self.ALIGN) * self.ALIGN
        self.buf = buf if buf is not None else torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)] if self.size > 0 else []   # (offset, bytes), by offset

    def _round(self, n: int) -> int:
        return max(self.ALIGN, -(-int(n) // self.ALIGN) * self.ALIGN)

    def alloc(self, nbytes: int):
        """(offset, a uint8 view of nbytes) of the first free block that fits, or None."""
        n = self._round(nbytes)
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, ln - n)
                return off, self.buf[off:off + int(nbytes)]
        return None

    def release(self, off: int, nbytes: int):
        n = self._round(nbytes)
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        if (i > 0 and self.free[i - 1][0] + self.free[i - 1][1] > off) or (i < len(self.free) and off + n > self.free[i][0]):
            raise ValueError("release of a block that overlaps free space")
        self.free.insert(i, (off, n))
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:       # merge with the next block
            self.free[i] = (off, n + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:     # and with the previous one
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def free_bytes(self) -> int:
        return sum(ln for _, ln in self.free)


@dataclass
class Request:
    rid: int
    grid: tpx.Grid
    geom: tpx.Geometry
    probe: tpx.Probe
    m: torch.Tensor
    d_obs: torch.Tensor
    arrival: float = 0.0          # seconds after the start of the run
    cancel_at: Optional[float] = None   # the client withdraws the request at this time (seconds)

    @property
    def updates(self) -> int:
        """Grid-point updates of one gradient (forward + adjoint, padded grid)."""
        npad = int(np.prod([s + 2 * self.grid.nbl for s in self.grid.shape]))
        return self.geom.nshots * npad * 2 * (self.grid.nt - 1)

    def workspace_bytes(self) -> int:
        return tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, self.grid, self.geom, self.probe)


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    g: Optional[torch.Tensor] = None
    J: Optional[torch.Tensor] = None
    status: str = "ok"

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req: Request, job: tpx.Job, stream, need: int, admitted: float, ws_off: int, ws_bytes: int):
        self.req, self.job, self.stream, self.need, self.admitted = req, job, stream, need, admitted
        self.ws_off, self.ws_bytes = ws_off, ws_bytes
        self.events = collections.deque()
        self.cancelled = False


class Server:
    """max_active defaults to 3, one fewer than the hardware queues HIP gives a
    process here (GPU_MAX_HW_QUEUES = 4).  Measured on a Poisson mix of 2D and
    3D requests: 3 jobs keep the saturated throughput of 4 and cut the p50 and
    p99 latencies under load; 2 lose the saturated gain; more than 4 share
    queues and caches and fall below the sequential path's throughput.

    A job whose levels hold at least `large_points` padded grid points over all
    its shots fills the GPU with one step launch by itself; at most `max_large`
    such jobs run at once (two interleave well, four slow each other down),
    while smaller jobs fill the gaps around them.  Waiting requests are
    admitted in arrival order, a blocked large request letting smaller ones
    behind it pass."""

    def __init__(self, hbm_budget_bytes: float = 200e9, chunk_steps: int = 64, max_active: int = 3,
                 nstreams: int = 8, inflight: int = 2, device=None, large_points: float = 3e6, max_large: int = 2):
        self.large_points = float(large_points)
        self.max_large = int(max_large)
        self.budget = float(hbm_budget_bytes)
        self.chunk = int(chunk_steps)
        self.max_active = int(max_active)
        self.inflight = int(inflight)
        self.device = torch.device(device or "cuda")
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(nstreams)]
        self.peak_active = 0
        self.peak_large = 0
        self.peak_bytes = 0
        self.in_use_bytes = 0   # workspace bytes still held when run() returns

    def run(self, requests: List[Request]) -> Dict[int, Result]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        pend = collections.deque(reqs)
        waiting = collections.deque()
        active: List[_Active] = []
        free_streams = list(self.streams)
        used = 0
        wsb: Dict[int, int] = {}   # workspace bytes per request (sizing builds the tables: done once)
        results: Dict[int, Result] = {}
        # the workspaces' arena: at most max_active jobs hold workspace at once, so
        # twice the largest max_active workspaces (slack for fragmentation), never
        # less than the largest one, never more than the budget
        for r in reqs:   # sizing builds the tables: before the clock starts
            wsb[r.rid] = r.workspace_bytes()
        sizes = sorted(wsb.values(), reverse=True)
        want = max(2 * sum(sizes[:self.max_active]), sizes[0] if sizes else 0) + Arena.ALIGN * self.max_active
        arena = Arena(min(self.budget, want), device=self.device)
        t0 = time.perf_counter()
        while pend or waiting or active:
            now = time.perf_counter() - t0
            while pend and pend[0].arrival <= now:
                r = pend.popleft()
                results[r.rid] = Result(r.rid, r.arrival)
                waiting.append(r)
            # withdrawn requests: a waiting one leaves the queue; an active one
            # stops advancing and frees its workspace once its queued chunks ran
            for r in [q for q in waiting if q.cancel_at is not None and q.cancel_at <= now]:
                waiting.remove(r)
                results[r.rid].status = "cancelled"
                results[r.rid].finished = now
            for st in active:
                if not st.cancelled and st.req.cancel_at is not None and st.req.cancel_at <= now:
                    st.cancelled = True
                    results[st.req.rid].status = "cancelled"
            # admission at chunk boundaries
            def need(req):
                if req.rid not in wsb:
                    wsb[req.rid] = req.workspace_bytes()
                return wsb[req.rid] + 4 * int(np.prod(req.grid.shape)) + 8

            nlarge = sum(1 for st in active if self._large(st.req))
            slots = min(self.max_active - len(active), len(free_streams))
            admit, reject = admission_plan(list(waiting), slots, self.budget - used, self.budget, nlarge,
                                           self.max_large, need, self._large)
            for req in reject:
                waiting.remove(req)
                results[req.rid].status = "rejected: workspace exceeds the HBM budget"
                results[req.rid].finished = now
            for req in admit:
                got = arena.alloc(wsb[req.rid])
                if got is None:
                    break   # fragmented: this request and the later ones wait for a release
                ws_off, ws = got
                waiting.remove(req)
                nlarge += 1 if self._large(req) else 0
                stream = free_streams.pop()
                # the job's inputs (m, d_obs) come from the caller's stream
                stream.wait_stream(torch.cuda.current_stream(self.device))
                with torch.cuda.stream(stream):
                    job = tpx.Job(req.grid, req.geom, req.probe, req.m, req.d_obs, ws=ws, stream=stream)
                active.append(_Active(req, job, stream, need(req), now, ws_off, wsb[req.rid]))
                results[req.rid].admitted = now
                used += need(req)
                self.peak_active = max(self.peak_active, len(active))
                self.peak_large = max(self.peak_large, nlarge)
                self.peak_bytes = max(self.peak_bytes, used)
            # advance every active job by one chunk, keeping a bounded queue per job
            for st in list(active):
                while st.events and st.events[0].query():
                    st.events.popleft()
                if st.job.finished or st.cancelled:
                    if not st.events:
                        res = results[st.req.rid]
                        res.finished = time.perf_counter() - t0
                        if not st.cancelled:
                            res.g, res.J = st.job.g, st.job.J
                        st.job.close()
                        st.job.ws = None
                        arena.release(st.ws_off, st.ws_bytes)   # its chunks have run
                        active.remove(st)
                        free_streams.append(st.stream)
                        used -= st.need
                    continue
                if len(st.events) < self.inflight:
                    st.job.advance(self.chunk, stream=st.stream)
                    ev = torch.cuda.Event()
                    ev.record(st.stream)
                    st.events.append(ev)
            if not active and waiting and not free_streams:
                raise RuntimeError("no stream available")
            if not active and not waiting and pend:
                time.sleep(max(0.0, min(pend[0].arrival - (time.perf_counter() - t0), 0.001)))
        torch.cuda.synchronize(self.device)
        self.in_use_bytes = used
        return results


    def _large(self, req: Request) -> bool:
        npad = int(np.prod([n + 2 * req.grid.nbl for n in req.grid.shape]))
        return req.geom.nshots * npad >= self.large_points


def run_sequential(requests: List[Request], device=None) -> Dict[int, Result]:
    """The plain path: one gradient call at a time, in arrival order."""
    device = torch.device(device or "cuda")
    reqs = sorted(requests, key=lambda r: r.arrival)
    results: Dict[int, Result] = {}
    stream = torch.cuda.current_stream(device)
    wsb = {q.rid: q.workspace_bytes() for q in reqs}   # sizing builds the tables: before the clock starts
    ws_all = torch.empty(max(list(wsb.values()) + [1]), dtype=torch.uint8, device=device)
    t0 = time.perf_counter()
    for req in reqs:
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        res = Result(req.rid, req.arrival, admitted=time.perf_counter() - t0)
        ws = ws_all[:wsb[req.rid]]
        g, J = tpx.gradient_probed(req.grid, req.geom, req.probe, req.m, req.d_obs, ws=ws, stream=stream)
        torch.cuda.synchronize(device)
        res.finished = time.perf_counter() - t0
        res.g, res.J = g, J
        results[req.rid] = res
    return results


def summarize(results: Dict[int, Result], requests: List[Request]) -> dict:
    ok = [r for r in results.values() if r.status == "ok"]
    cancelled = sum(1 for r in results.values() if r.status == "cancelled")
    lat = np.array([r.latency for r in ok]) * 1e3
    start = min(r.arrival for r in results.values())
    end = max(r.finished for r in ok)
    upd = sum(q.updates for q in requests if results[q.rid].status == "ok")
    return {"requests": len(results), "completed": len(ok), "cancelled": cancelled,
            "rejected": len(results) - len(ok) - cancelled,
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_ms": round(float(lat.mean()), 2), "makespan_s": round(end - start, 3),
            "gpts_per_s": round(upd / (end - start) / 1e9, 2)}


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n)) - 0.0
