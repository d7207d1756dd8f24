"""FP64 CPU oracle for the probed adjoint-state FWI gradient.

TEST INFRASTRUCTURE ONLY: the slow, plain reference that the GPU library is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this package; the product path never does.  It shares
no code with the HIP library (``paper_2104_00794_amd``) and imports nothing
from it.

The arithmetic lives in ``tpx_oracle.c`` (plain C, double precision); this
module only builds it with gcc and marshals NumPy arrays through ctypes.

Paper sections followed (Louboutin & Herrmann, arXiv 2104.00794):
  * misfit 0.5 ||F(m;q) - d_obs||^2 ............ Methodology, Eq. (2)
  * exact gradient sum_t  u_tt[t] v[t] ......... Methodology, Eq. (3)
  * probed gradient (1/r) tr((Q^T u_tt)(v^T Q)) . Methodology, Eq. (4), Algorithm 1
  * probes: Rademacher / Gaussian ............. Randomized trace estimation, Eq. (1)
  * probes from the data's range, Q = qr(D D^T Z) . Choice of the probing matrix Q, Eq. (6)

Parity status: all functions are pinned by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force and NumPy's Philox known-answer vectors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpx_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "liboracle.so")

PROBE_RADEMACHER = 0
PROBE_GAUSS_B64 = 1
PROBE_IDENTITY = 2
PROBE_EXPLICIT = 3

_KINDS = {"rademacher": PROBE_RADEMACHER, "gauss_b64": PROBE_GAUSS_B64,
          "identity": PROBE_IDENTITY, "explicit": PROBE_EXPLICIT}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    os.makedirs(_BUILD_DIR, exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("nbl", ctypes.c_int32), ("order", ctypes.c_int32), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("damp_vmax", ctypes.c_double), ("damp_R", ctypes.c_double)]


class _Geom(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("src_pos", ctypes.POINTER(ctypes.c_double)), ("rec_pos", ctypes.POINTER(ctypes.c_double)),
                ("wavelet", ctypes.POINTER(ctypes.c_double))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        lib.orc_forward.argtypes = [P(_Grid), P(_Geom), dp, dp, dp]
        lib.orc_adjoint.argtypes = [P(_Grid), P(_Geom), dp, dp, dp, dp]
        lib.orc_gradient_full.argtypes = [P(_Grid), P(_Geom), dp, dp, ctypes.c_int32, dp, dp, dp]
        lib.orc_gradient_probed.argtypes = [P(_Grid), P(_Geom), dp, dp, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_uint64, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                            P(ctypes.c_int64), ctypes.c_int64, dp, dp, dp]
        lib.orc_probe_matrix.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32, dp]
        lib.orc_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        lib.orc_laplacian.argtypes = [P(_Grid), dp, dp]
        lib.orc_pad_model.argtypes = [P(_Grid), dp, dp]
        lib.orc_damping.argtypes = [P(_Grid), dp]
        lib.orc_propagate_field.argtypes = [P(_Grid), dp, dp, dp]
        for name in ("orc_forward", "orc_adjoint", "orc_gradient_full", "orc_gradient_probed",
                     "orc_probe_matrix", "orc_propagate_field"):
            getattr(lib, name).restype = ctypes.c_int
        lib.orc_laplacian.restype = None
        lib.orc_pad_model.restype = None
        lib.orc_damping.restype = None
        lib.orc_philox4x64_10.restype = None
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


_ERRS = {1: "invalid argument", 2: "source or receiver outside the grid", 3: "out of host memory"}


def _check(rc: int):
    if rc != 0:
        raise OracleError(_ERRS.get(rc, "error %d" % rc))


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Regular grid: physical nodes ``shape`` = (nz, nx) in 2D or (nz, ny, nx) in 3D."""
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
        g.n[0], g.n[1], g.n[2] = nx, ny, nz
        g.h, g.nbl, g.order, g.dt, g.nt = self.h, self.nbl, self.order, self.dt, self.nt
        g.damp_vmax, g.damp_R = self.damp_vmax, self.damp_R
        return g

    @property
    def padded_shape(self):
        if self.ndim == 2:
            return (self.shape[0] + 2 * self.nbl, self.shape[1] + 2 * self.nbl)
        return tuple(s + 2 * self.nbl for s in self.shape)


class _GeomHolder:
    def __init__(self, src_pos, rec_pos, wavelet):
        self.src = np.ascontiguousarray(src_pos, dtype=np.float64).reshape(-1, 3)
        S = self.src.shape[0]
        self.rec = np.ascontiguousarray(rec_pos, dtype=np.float64).reshape(S, -1, 3)
        self.wav = np.ascontiguousarray(wavelet, dtype=np.float64).reshape(S, -1)
        self.c = _Geom()
        self.c.nshots = S
        self.c.nrec = self.rec.shape[1]
        self.c.src_pos = _dp(self.src)
        self.c.rec_pos = _dp(self.rec) if self.rec.size else None
        self.c.wavelet = _dp(self.wav)


def _m(grid: Grid, m) -> np.ndarray:
    a = np.ascontiguousarray(m, dtype=np.float64)
    assert a.shape == tuple(grid.shape), (a.shape, grid.shape)
    return a


def forward(grid: Grid, m, src_pos, rec_pos, wavelet, return_history: bool = False):
    """Traces d[S][nt][nrec] = F(m; q); optionally u^k on the physical grid."""
    lib = _load()
    geo = _GeomHolder(src_pos, rec_pos, wavelet)
    S, nrec = geo.c.nshots, geo.c.nrec
    d = np.zeros((S, grid.nt, nrec))
    hist = np.zeros((S, grid.nt) + tuple(grid.shape)) if return_history else None
    _check(lib.orc_forward(ctypes.byref(grid.c()), ctypes.byref(geo.c), _dp(_m(grid, m)), _dp(d), _dp(hist)))
    return (d, hist) if return_history else d


def adjoint(grid: Grid, m, src_pos, rec_pos, d_in, return_history: bool = False):
    """q_adj[S][nt] = F^T d_in; optionally lambda^k on the physical grid."""
    lib = _load()
    S = np.asarray(src_pos).reshape(-1, 3).shape[0]
    geo = _GeomHolder(src_pos, rec_pos, np.zeros((S, grid.nt)))
    S = geo.c.nshots
    din = np.ascontiguousarray(d_in, dtype=np.float64)
    q = np.zeros((S, grid.nt))
    hist = np.zeros((S, grid.nt) + tuple(grid.shape)) if return_history else None
    _check(lib.orc_adjoint(ctypes.byref(grid.c()), ctypes.byref(geo.c), _dp(_m(grid, m)), _dp(din), _dp(q),
                           _dp(hist)))
    return (q, hist) if return_history else q


def gradient_full(grid: Grid, m, src_pos, rec_pos, wavelet, d_obs, form: int = 0, return_traces=False):
    """Exact gradient (Eq. 3) with the full forward history; returns (g, J)."""
    lib = _load()
    geo = _GeomHolder(src_pos, rec_pos, wavelet)
    dobs = np.ascontiguousarray(d_obs, dtype=np.float64)
    g = np.zeros(tuple(grid.shape))
    J = np.zeros(1)
    dout = np.zeros((geo.c.nshots, grid.nt, geo.c.nrec)) if return_traces else None
    _check(lib.orc_gradient_full(ctypes.byref(grid.c()), ctypes.byref(geo.c), _dp(_m(grid, m)), _dp(dobs),
                                 form, _dp(g), _dp(J), _dp(dout)))
    if return_traces:
        return g, float(J[0]), dout
    return g, float(J[0])


def gradient_probed(grid: Grid, m, src_pos, rec_pos, wavelet, d_obs, kind="rademacher", r=8, seed=0,
                    Z=None, scale=1.0, side=0, imaging=0, points=None, return_traces=False):
    """Probed gradient (Eq. 4, Algorithm 1); returns (g~, J).

    ``imaging``: 0 images the probed fields pointwise (Eq. 4); 1 takes the
    inner product of their centred spatial gradients (Eq. 5 with D_x = grad;
    zero on the outermost physical nodes).
    ``points``: optional flat physical indices; then g~ is returned only there.
    """
    lib = _load()
    geo = _GeomHolder(src_pos, rec_pos, wavelet)
    kind_id = _KINDS[kind] if isinstance(kind, str) else int(kind)
    dobs = np.ascontiguousarray(d_obs, dtype=np.float64)
    Zc = None
    if kind_id == PROBE_EXPLICIT:
        Zc = np.ascontiguousarray(Z, dtype=np.float64).reshape(geo.c.nshots, grid.nt, r)
    if points is not None:
        pts = np.ascontiguousarray(points, dtype=np.int64)
        g = np.zeros(pts.shape[0])
        pp, npts = pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pts.shape[0]
    else:
        g = np.zeros(tuple(grid.shape))
        pp, npts = None, 0
    J = np.zeros(1)
    dout = np.zeros((geo.c.nshots, grid.nt, geo.c.nrec)) if return_traces else None
    _check(lib.orc_gradient_probed(ctypes.byref(grid.c()), ctypes.byref(geo.c), _dp(_m(grid, m)), _dp(dobs),
                                   kind_id, r, ctypes.c_uint64(seed), _dp(Zc), float(scale), side, imaging, pp, npts,
                                   _dp(g), _dp(J), _dp(dout)))
    if return_traces:
        return g, float(J[0]), dout
    return g, float(J[0])


def range_finder_probes(d_obs, r: int, seed: int) -> np.ndarray:
    """Probing matrices that capture the range of the data's time covariance
    (Choice of the probing matrix Q, Eq. 6): per shot, the observed traces form
    D (nt x nrec), A = D D^T, and Q is the orthonormal factor of the reduced QR
    of A Z, with Z that shot's Rademacher probing matrix (same seed and counter
    as ``probe_matrix``).  Returns Q as [S][nt][r]; it is used with c = 1."""
    D = np.asarray(d_obs, dtype=np.float64)
    S, nt, nrec = D.shape
    Q = np.empty((S, nt, r))
    for s in range(S):
        Z = probe_matrix("rademacher", r, seed, nt, s)
        Y = D[s] @ (D[s].T @ Z)   # A Z, with A applied in factored form
        Q[s] = np.linalg.qr(Y, mode="reduced")[0]
    return Q


def probe_matrix(kind, r: int, seed: int, nt: int, shot: int) -> np.ndarray:
    lib = _load()
    kind_id = _KINDS[kind] if isinstance(kind, str) else int(kind)
    Z = np.zeros((nt, r))
    _check(lib.orc_probe_matrix(kind_id, r, ctypes.c_uint64(seed), nt, shot, _dp(Z)))
    return Z


def philox4x64_10(counter, key):
    lib = _load()
    c = (ctypes.c_uint64 * 4)(*[int(x) % 2**64 for x in counter])
    k = (ctypes.c_uint64 * 2)(*[int(x) % 2**64 for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib.orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def laplacian(grid: Grid, u_pad) -> np.ndarray:
    lib = _load()
    u = np.ascontiguousarray(u_pad, dtype=np.float64)
    assert u.shape == grid.padded_shape
    out = np.zeros_like(u)
    lib.orc_laplacian(ctypes.byref(grid.c()), _dp(u), _dp(out))
    return out


def pad_model(grid: Grid, m) -> np.ndarray:
    lib = _load()
    out = np.zeros(grid.padded_shape)
    lib.orc_pad_model(ctypes.byref(grid.c()), _dp(_m(grid, m)), _dp(out))
    return out


def damping(grid: Grid) -> np.ndarray:
    lib = _load()
    out = np.zeros(grid.padded_shape)
    lib.orc_damping(ctypes.byref(grid.c()), _dp(out))
    return out


def propagate_field(grid: Grid, m, f) -> np.ndarray:
    """Manufactured-solution hook: u^{nt-1} for a distributed source f[k][padded]."""
    lib = _load()
    fa = np.ascontiguousarray(f, dtype=np.float64)
    assert fa.shape == (grid.nt - 1,) + grid.padded_shape
    out = np.zeros(grid.padded_shape)
    _check(lib.orc_propagate_field(ctypes.byref(grid.c()), _dp(_m(grid, m)), _dp(fa), _dp(out)))
    return out
