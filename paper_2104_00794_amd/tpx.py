"""Thin Python binding of the HIP library ``libtpx.so`` (C-ABI: include/tpx.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI.  PyTorch supplies device memory (inputs, outputs and
the workspace) and the current stream.  If the library has not been built the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libtpx.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "tpx.h")

OK, E_INVAL, E_CFL, E_GEOM, E_NOMEM, E_DEVICE, E_NUMERIC, E_STATE = range(8)
STATUS_NAMES = {0: "TPX_OK", 1: "TPX_E_INVAL", 2: "TPX_E_CFL", 3: "TPX_E_GEOM", 4: "TPX_E_NOMEM",
                5: "TPX_E_DEVICE", 6: "TPX_E_NUMERIC", 7: "TPX_E_STATE"}

CALL_FORWARD, CALL_ADJOINT, CALL_GRADIENT_PROBED, CALL_GRADIENT_FULL, CALL_FORWARD_PROBED, \
    CALL_BACKWARD_PROBED, CALL_RANGE_FINDER, CALL_OBJECTIVE = range(8)

PROBE_KINDS = {"rademacher": 0, "gauss_b64": 1, "identity": 2, "explicit": 3, "range_finder": 4}


class TpxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("nbl", ctypes.c_int32), ("space_order", ctypes.c_int32), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("damp_vmax", ctypes.c_double), ("damp_R", ctypes.c_double)]


class _Geom(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("src_pos", ctypes.POINTER(ctypes.c_double)), ("rec_pos", ctypes.POINTER(ctypes.c_double)),
                ("wavelet", ctypes.c_void_p)]


class _Probe(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("r", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("Z", ctypes.c_void_p), ("scale", ctypes.c_double), ("block", ctypes.c_int32),
                ("keep_vbar", ctypes.c_int32), ("dtt_side", ctypes.c_int32), ("imaging", ctypes.c_int32)]


_lib = None


def exported_names_in_header(path: str = HEADER) -> list:
    """Function names the public header declares."""
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpx_[a-z_]+)\s*\(", src)))


def lib():
    """Load libtpx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtpx.so is not built (python -m paper_2104_00794_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.tpx_last_error.restype = ctypes.c_char_p
    L.tpx_version.restype = ctypes.c_char_p
    L.tpx_workspace_bytes.argtypes = [i32, P(_Grid), P(_Geom), P(_Probe)]
    L.tpx_workspace_bytes.restype = sz
    L.tpx_state_bytes.argtypes = [P(_Grid), P(_Geom), P(_Probe)]
    L.tpx_state_bytes.restype = sz
    L.tpx_forward.argtypes = [P(_Grid), P(_Geom), vp, vp, vp, sz, vp]
    L.tpx_adjoint.argtypes = [P(_Grid), P(_Geom), vp, vp, vp, vp, sz, vp]
    L.tpx_objective.argtypes = [P(_Grid), P(_Geom), vp, vp, vp, vp, vp, sz, vp]
    L.tpx_gradient_probed.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, vp, vp, vp, sz, vp]
    L.tpx_gradient_full.argtypes = [P(_Grid), P(_Geom), vp, vp, vp, vp, vp, vp, sz, vp]
    L.tpx_gradient_probed_noalloc.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, vp, vp, vp]
    L.tpx_forward_probed.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, sz, vp, sz, vp]
    L.tpx_backward_probed.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, sz, vp, vp, sz, vp]
    L.tpx_probe_matrix.argtypes = [P(_Probe), i32, i32, vp, vp]
    L.tpx_range_finder_probes.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, sz, vp]
    L.tpx_check_workspace.argtypes = [vp, vp]
    L.tpx_job_create.argtypes = [P(_Grid), P(_Geom), P(_Probe), vp, vp, vp, vp, vp, vp, sz, vp,
                                 P(ctypes.c_void_p)]
    L.tpx_job_advance.argtypes = [vp, i32, vp, P(i32)]
    L.tpx_job_progress.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    L.tpx_job_destroy.argtypes = [vp]
    L.tpx_job_destroy.restype = None
    L.tpx_set_option.argtypes = [i32, ctypes.c_int64]
    L.tpx_set_option.restype = ctypes.c_int
    L.tpx_get_option.argtypes = [i32]
    L.tpx_get_option.restype = ctypes.c_int64
    L.tpx_profile_enable.argtypes = [i32]
    L.tpx_profile_enable.restype = None
    L.tpx_profile_read.argtypes = [i32, P(ctypes.c_double), P(ctypes.c_int64)]
    for name in ("tpx_forward", "tpx_objective", "tpx_adjoint", "tpx_gradient_probed", "tpx_gradient_full",
                 "tpx_gradient_probed_noalloc",
                 "tpx_forward_probed", "tpx_backward_probed", "tpx_probe_matrix", "tpx_check_workspace", "tpx_profile_read",
                 "tpx_job_create", "tpx_job_advance", "tpx_job_progress"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise TpxError(status, lib().tpx_last_error().decode())


# --------------------------------------------------------------------------- #
# problem description
# --------------------------------------------------------------------------- #

@dataclass
class Grid:
    """Physical nodes ``shape`` = (nz, nx) in 2D or (nz, ny, nx) in 3D."""
    shape: Sequence[int]
    h: float
    dt: float
    nt: int
    order: int = 8
    nbl: int = 20
    damp_vmax: float = 4.5
    damp_R: float = 1e-3

    @property
    def ndim(self) -> int:
        return len(self.shape)

    def c(self) -> _Grid:
        g = _Grid()
        g.ndim = self.ndim
        if self.ndim == 2:
            nz, nx = self.shape
            ny = 1
        else:
            nz, ny, nx = self.shape
        g.n[0], g.n[1], g.n[2] = int(nx), int(ny), int(nz)
        g.h, g.nbl, g.space_order, g.dt, g.nt = float(self.h), int(self.nbl), int(self.order), float(self.dt), \
            int(self.nt)
        g.damp_vmax, g.damp_R = float(self.damp_vmax), float(self.damp_R)
        return g


class Geometry:
    """Sources, receivers (host float64 positions in m) and device wavelets."""

    def __init__(self, src_pos, rec_pos, wavelet=None):
        self.src = np.ascontiguousarray(src_pos, dtype=np.float64).reshape(-1, 3)
        S = self.src.shape[0]
        self.rec = np.ascontiguousarray(rec_pos, dtype=np.float64).reshape(S, -1, 3)
        self.wavelet = wavelet
        if wavelet is not None:
            assert wavelet.dtype.is_floating_point and wavelet.is_contiguous() and wavelet.shape[0] == S

    @property
    def nshots(self) -> int:
        return self.src.shape[0]

    @property
    def nrec(self) -> int:
        return self.rec.shape[1]

    def c(self) -> _Geom:
        g = _Geom()
        g.nshots = self.nshots
        g.nrec = self.nrec
        g.src_pos = self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.rec_pos = self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self.rec.size else None
        g.wavelet = self.wavelet.data_ptr() if self.wavelet is not None else None
        return g


@dataclass
class Probe:
    kind: str = "rademacher"
    r: int = 8
    seed: int = 0
    Z: Optional[object] = None       # device tensor [S][nt][r] for kind="explicit"
    scale: float = 1.0
    block: int = 0
    keep_vbar: bool = False
    dtt_side: int = 0                # 1: the second time difference on the forward side (Algorithm 1)
    imaging: int = 0                 # 1: gradient inner product of the probed fields (Eq. 5); keep_vbar=True

    def c(self) -> _Probe:
        p = _Probe()
        p.kind = PROBE_KINDS[self.kind]
        p.r = int(self.r)
        p.seed = int(self.seed) % 2 ** 64
        p.Z = self.Z.data_ptr() if self.Z is not None else None
        p.scale = float(self.scale)
        p.block = int(self.block)
        p.keep_vbar = 1 if self.keep_vbar else 0
        p.dtt_side = int(self.dtt_side)
        p.imaging = int(self.imaging)
        return p


# --------------------------------------------------------------------------- #
# calls
# --------------------------------------------------------------------------- #

def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _use_on(stream, *tensors):
    """The library reads and writes `tensors` on `stream`.  When that is not
    the current stream (on which PyTorch's caching allocator may have placed
    them), mark them in use there, so their memory is not handed to another
    allocation before `stream` has finished with it."""
    if stream is None:
        return
    torch = _torch()
    if stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _dev_f32(t, shape=None, name="tensor"):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def workspace_bytes(call: int, grid: Grid, geom: Geometry, probe: Optional[Probe] = None) -> int:
    g, ge = grid.c(), geom.c()
    p = probe.c() if probe is not None else None
    n = lib().tpx_workspace_bytes(call, ctypes.byref(g), ctypes.byref(ge), ctypes.byref(p) if p else None)
    if n == 0:
        raise TpxError(E_INVAL, lib().tpx_last_error().decode())
    return int(n)


def state_bytes(grid: Grid, geom: Geometry, probe: Probe) -> int:
    g, ge, p = grid.c(), geom.c(), probe.c()
    n = lib().tpx_state_bytes(ctypes.byref(g), ctypes.byref(ge), ctypes.byref(p))
    if n == 0:
        raise TpxError(E_INVAL, lib().tpx_last_error().decode())
    return int(n)


def alloc_workspace(call: int, grid: Grid, geom: Geometry, probe: Optional[Probe] = None, device=None):
    """A caller-owned device workspace of the size the call needs."""
    torch = _torch()
    n = workspace_bytes(call, grid, geom, probe)
    try:
        return torch.empty(n, dtype=torch.uint8, device=device or "cuda")
    except torch.cuda.OutOfMemoryError as e:
        raise TpxError(E_NOMEM, "cannot allocate a %d-byte workspace: %s" % (n, e)) from None


def _ws(ws, call, grid, geom, probe, device):
    if ws is None:
        ws = alloc_workspace(call, grid, geom, probe, device)
    return ws


def check_workspace(ws, stream=None):
    _check(lib().tpx_check_workspace(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(_stream(stream))))


def forward(grid: Grid, geom: Geometry, m, ws=None, stream=None):
    """Traces d[S][nt][nrec] = F(m; q)."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    d = torch.empty((geom.nshots, grid.nt, geom.nrec), dtype=torch.float32, device=m.device)
    ws = _ws(ws, CALL_FORWARD, grid, geom, None, m.device)
    g, ge = grid.c(), geom.c()
    _use_on(stream, m, d, ws)
    _check(lib().tpx_forward(ctypes.byref(g), ctypes.byref(ge), m.data_ptr(), d.data_ptr(), ws.data_ptr(),
                             ws.numel(), _stream(stream)))
    return d


def objective(grid: Grid, geom: Geometry, m, d_obs, ws=None, stream=None, J_out=None, return_traces: bool = False):
    """J = 1/2 ||F(m) - d_obs||^2 (Eq. 2) as a device double [1]: returns J[, d]."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
    J = J_out if J_out is not None else torch.empty(1, dtype=torch.float64, device=m.device)
    d = torch.empty((geom.nshots, grid.nt, geom.nrec), dtype=torch.float32, device=m.device) if return_traces \
        else None
    ws = _ws(ws, CALL_OBJECTIVE, grid, geom, None, m.device)
    g, ge = grid.c(), geom.c()
    _use_on(stream, m, d_obs, J, d, ws)
    _check(lib().tpx_objective(ctypes.byref(g), ctypes.byref(ge), m.data_ptr(), d_obs.data_ptr(), J.data_ptr(),
                               d.data_ptr() if d is not None else None, ws.data_ptr(), ws.numel(), _stream(stream)))
    return (J, d) if return_traces else J


def adjoint(grid: Grid, geom: Geometry, m, d_in, ws=None, stream=None):
    """q_adj[S][nt] = F^T d_in."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    _dev_f32(d_in, (geom.nshots, grid.nt, geom.nrec), "d_in")
    q = torch.empty((geom.nshots, grid.nt), dtype=torch.float32, device=m.device)
    ws = _ws(ws, CALL_ADJOINT, grid, geom, None, m.device)
    g, ge = grid.c(), geom.c()
    _use_on(stream, m, d_in, q, ws)
    _check(lib().tpx_adjoint(ctypes.byref(g), ctypes.byref(ge), m.data_ptr(), d_in.data_ptr(), q.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(stream)))
    return q


def gradient_probed(grid: Grid, geom: Geometry, probe: Probe, m, d_obs, ws=None, stream=None,
                    return_traces: bool = False, g_out=None, J_out=None):
    """Probed gradient (Eq. 4 / Algorithm 1): returns (g, J[, d])."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
    g = g_out if g_out is not None else torch.empty(tuple(grid.shape), dtype=torch.float32, device=m.device)
    J = J_out if J_out is not None else torch.empty(1, dtype=torch.float64, device=m.device)
    d = torch.empty((geom.nshots, grid.nt, geom.nrec), dtype=torch.float32, device=m.device) if return_traces \
        else None
    ws = _ws(ws, CALL_GRADIENT_PROBED, grid, geom, probe, m.device)
    gc, ge, pc = grid.c(), geom.c(), probe.c()
    _use_on(stream, m, d_obs, g, J, d, ws, probe.Z)
    _check(lib().tpx_gradient_probed(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), m.data_ptr(),
                                     d_obs.data_ptr(), g.data_ptr(), J.data_ptr(),
                                     d.data_ptr() if d is not None else None, ws.data_ptr(), ws.numel(),
                                     _stream(stream)))
    return (g, J, d) if return_traces else (g, J)


NOALLOC_SCRATCH_BYTES = 64 << 20


def gradient_probed_noalloc(grid: Grid, geom: Geometry, probe: Probe, m, d_obs, g_out, J_out, stream=None,
                            d_out=None):
    """The probed gradient through the allocation-free entry point: the
    library's static per-GPU scratch is the workspace, and the caller passes
    every output (g_out, J_out, optionally d_out)."""
    _dev_f32(m, grid.shape, "m")
    _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
    _dev_f32(g_out, grid.shape, "g_out")
    torch = _torch()
    if not (isinstance(J_out, torch.Tensor) and J_out.is_cuda and J_out.dtype == torch.float64 and J_out.numel() >= 1):
        raise TypeError("J_out must be a float64 CUDA tensor with at least one element")
    if d_out is not None:
        _dev_f32(d_out, (geom.nshots, grid.nt, geom.nrec), "d_out")
    gc, ge, pc = grid.c(), geom.c(), probe.c()
    _use_on(stream, m, d_obs, g_out, J_out, d_out, probe.Z)
    _check(lib().tpx_gradient_probed_noalloc(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), m.data_ptr(),
                                             d_obs.data_ptr(), g_out.data_ptr(), J_out.data_ptr(),
                                             d_out.data_ptr() if d_out is not None else None, _stream(stream)))
    return g_out, J_out


def gradient_full(grid: Grid, geom: Geometry, m, d_obs, ws=None, stream=None, return_traces: bool = False):
    """Exact gradient (Eq. 3) from the stored forward history: returns (g, J[, d])."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
    g = torch.empty(tuple(grid.shape), dtype=torch.float32, device=m.device)
    J = torch.empty(1, dtype=torch.float64, device=m.device)
    d = torch.empty((geom.nshots, grid.nt, geom.nrec), dtype=torch.float32, device=m.device) if return_traces \
        else None
    ws = _ws(ws, CALL_GRADIENT_FULL, grid, geom, None, m.device)
    gc, ge = grid.c(), geom.c()
    _use_on(stream, m, d_obs, g, J, d, ws)
    _check(lib().tpx_gradient_full(ctypes.byref(gc), ctypes.byref(ge), m.data_ptr(), d_obs.data_ptr(),
                                   g.data_ptr(), J.data_ptr(), d.data_ptr() if d is not None else None,
                                   ws.data_ptr(), ws.numel(), _stream(stream)))
    return (g, J, d) if return_traces else (g, J)


def forward_probed(grid: Grid, geom: Geometry, probe: Probe, m, ws=None, state=None, stream=None):
    """Forward pass with probing: returns (d, state) where state holds ubar."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    d = torch.empty((geom.nshots, grid.nt, geom.nrec), dtype=torch.float32, device=m.device)
    if state is None:
        state = torch.empty(state_bytes(grid, geom, probe), dtype=torch.uint8, device=m.device)
    ws = _ws(ws, CALL_FORWARD_PROBED, grid, geom, probe, m.device)
    gc, ge, pc = grid.c(), geom.c(), probe.c()
    _use_on(stream, m, d, state, ws, probe.Z)
    _check(lib().tpx_forward_probed(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), m.data_ptr(),
                                    d.data_ptr(), state.data_ptr(), state.numel(), ws.data_ptr(), ws.numel(),
                                    _stream(stream)))
    return d, state


def backward_probed(grid: Grid, geom: Geometry, probe: Probe, m, grad_d, state, ws=None, stream=None):
    """Back-propagation of grad_d with probed imaging against the stored ubar."""
    torch = _torch()
    _dev_f32(m, grid.shape, "m")
    _dev_f32(grad_d, (geom.nshots, grid.nt, geom.nrec), "grad_d")
    g = torch.empty(tuple(grid.shape), dtype=torch.float32, device=m.device)
    ws = _ws(ws, CALL_BACKWARD_PROBED, grid, geom, probe, m.device)
    gc, ge, pc = grid.c(), geom.c(), probe.c()
    _use_on(stream, m, grad_d, state, g, ws, probe.Z)
    _check(lib().tpx_backward_probed(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), m.data_ptr(),
                                     grad_d.data_ptr(), state.data_ptr(), state.numel(), g.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream(stream)))
    return g


def range_finder_probes(grid: Grid, geom: Geometry, probe: Probe, d_obs, ws=None, stream=None):
    """Q[S][nt][r] = qr(D D^T Z) per shot from the observed traces (Eq. 6); pass
    it as ``Probe(kind="explicit", Z=Q, scale=1)`` to the split forward/backward."""
    torch = _torch()
    _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
    Q = torch.empty((geom.nshots, grid.nt, probe.r), dtype=torch.float32, device=d_obs.device)
    ws = _ws(ws, CALL_RANGE_FINDER, grid, geom, probe, d_obs.device)
    gc, ge, pc = grid.c(), geom.c(), probe.c()
    _use_on(stream, d_obs, Q, ws)
    _check(lib().tpx_range_finder_probes(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), d_obs.data_ptr(),
                                         Q.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return Q


def probe_matrix(probe: Probe, nt: int, shot: int, device=None, stream=None):
    """Z[nt][r] of one shot, generated on the GPU."""
    torch = _torch()
    Z = torch.empty((nt, probe.r), dtype=torch.float32, device=device or "cuda")
    pc = probe.c()
    _use_on(stream, Z)
    _check(lib().tpx_probe_matrix(ctypes.byref(pc), int(nt), int(shot), Z.data_ptr(), _stream(stream)))
    return Z


class Job:
    """A probed-gradient job advanced a bounded number of time steps at a time.

    The caller owns every buffer (model, data, outputs, workspace); they are
    kept referenced here until the job is closed.
    """

    def __init__(self, grid: Grid, geom: Geometry, probe: Probe, m, d_obs, ws=None, stream=None, g=None, J=None):
        torch = _torch()
        _dev_f32(m, grid.shape, "m")
        _dev_f32(d_obs, (geom.nshots, grid.nt, geom.nrec), "d_obs")
        self.grid, self.geom, self.probe, self.m, self.d_obs = grid, geom, probe, m, d_obs
        self.g = g if g is not None else torch.empty(tuple(grid.shape), dtype=torch.float32, device=m.device)
        self.J = J if J is not None else torch.empty(1, dtype=torch.float64, device=m.device)
        self.ws = _ws(ws, CALL_GRADIENT_PROBED, grid, geom, probe, m.device)
        gc, ge, pc = grid.c(), geom.c(), probe.c()
        h = ctypes.c_void_p()
        _use_on(stream, m, d_obs, self.g, self.J, self.ws, probe.Z)
        _check(lib().tpx_job_create(ctypes.byref(gc), ctypes.byref(ge), ctypes.byref(pc), m.data_ptr(),
                                    d_obs.data_ptr(), self.g.data_ptr(), self.J.data_ptr(), None,
                                    self.ws.data_ptr(), self.ws.numel(), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.finished = False

    def advance(self, max_steps: int, stream=None) -> bool:
        """Enqueue up to max_steps time steps; True once all work is enqueued."""
        fin = ctypes.c_int32(0)
        _use_on(stream, self.m, self.d_obs, self.g, self.J, self.ws, self.probe.Z)
        _check(lib().tpx_job_advance(self._h, int(max_steps), _stream(stream), ctypes.byref(fin)))
        self.finished = bool(fin.value)
        return self.finished

    def progress(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tpx_job_progress(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        if self._h:
            lib().tpx_job_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


KERNEL_STEP, KERNEL_ACCUM_FWD, KERNEL_ACCUM_ADJ, KERNEL_ACCUM_FULL, KERNEL_STEP2, KERNEL_STEP3 = range(6)
OPT_OVERLAP_CONTRACTIONS = 1
OPT_MATRIX_CORES = 2
OPT_FUSED_STEPS_3D = 3
OPT_STEPS_2D = 4


def set_option(option: int, value: int):
    """Library-wide option (changes workspace sizes: set before sizing)."""
    _check(lib().tpx_set_option(int(option), int(value)))


def get_option(option: int) -> int:
    return int(lib().tpx_get_option(int(option)))


def profile_enable(on: bool):
    """Bracket every kernel launch with HIP events (for measurement runs)."""
    lib().tpx_profile_enable(1 if on else 0)


def profile_read(kind: int):
    """(total_ms, launches) of one kernel kind since profiling was enabled."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().tpx_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def version() -> str:
    return lib().tpx_version().decode()
