"""CPU tests of the C-ABI library: it loads, exports every symbol the public
header declares, and rejects bad arguments on the host before any launch."""
import ctypes

import numpy as np
import pytest

from tests.helpers import ensure_built

ensure_built()

from paper_2104_00794_amd import tpx  # noqa: E402


def _geom(src, rec):
    return tpx.Geometry(np.array(src, float), np.array(rec, float))


def test_library_exports_every_header_symbol():
    L = tpx.lib()
    names = tpx.exported_names_in_header()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert tpx.version().startswith("tpx")


GRID = dict(shape=(30, 40), h=10.0, dt=1.5, nt=100, order=8, nbl=5, damp_vmax=3.0)


def _call_forward(grid, geom, ws_bytes=1 << 40):
    # fake device pointers: validation fails on the host before anything is launched
    L = tpx.lib()
    g, ge = grid.c(), geom.c()
    ge.wavelet = 0x1000
    return L.tpx_forward(ctypes.byref(g), ctypes.byref(ge), 0x1000, 0x2000, 0x3000, ws_bytes, None)


def test_cfl_rejected():
    grid = tpx.Grid(**dict(GRID, dt=2.0))  # limit for order 8, 2D: 0.5546 * h / vmax = 1.849 ms
    st = _call_forward(grid, _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]]))
    assert st == tpx.E_CFL
    assert "stability" in tpx.lib().tpx_last_error().decode()


def test_geometry_outside_grid_rejected():
    grid = tpx.Grid(**GRID)
    st = _call_forward(grid, _geom([[100.0, 0, 50.0]], [[[400.0, 0, 20.0]]]))  # x max is 390 m
    assert st == tpx.E_GEOM
    st = _call_forward(grid, _geom([[-1.0, 0, 50.0]], [[[10.0, 0, 20.0]]]))
    assert st == tpx.E_GEOM


def test_workspace_too_small_rejected():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])
    need = tpx.workspace_bytes(tpx.CALL_FORWARD, grid, geom)
    assert _call_forward(grid, geom, ws_bytes=need - 1) == tpx.E_NOMEM


@pytest.mark.parametrize("bad", [dict(order=6), dict(nt=1), dict(h=0.0), dict(nbl=-1), dict(damp_R=0.0)])
def test_invalid_grid_rejected(bad):
    grid = tpx.Grid(**dict(GRID, **bad))
    assert _call_forward(grid, _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])) == tpx.E_INVAL


def test_workspace_bytes_by_call():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0], [200.0, 0, 50.0]], [[[10.0, 0, 20.0]] * 3] * 2)
    p = tpx.Probe(r=8)
    fwd = tpx.workspace_bytes(tpx.CALL_FORWARD, grid, geom)
    prb = tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, p)
    full = tpx.workspace_bytes(tpx.CALL_GRADIENT_FULL, grid, geom)
    assert 0 < fwd < prb and fwd < full
    # identity probes need r == nt
    with pytest.raises(tpx.TpxError):
        tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(kind="identity", r=8))
    # probe accumulators are S * r * N_phys floats
    assert tpx.state_bytes(grid, geom, p) >= 2 * 8 * 30 * 40 * 4


def test_full_history_of_3d_config_exceeds_one_gpu():
    # 401 x 401 x 301 nodes, nt = 2001: the stored forward history alone is > 288 GB
    grid = tpx.Grid((301, 401, 401), h=12.5, dt=1.25, nt=2001, order=8, nbl=20, damp_vmax=4.0)
    geom = _geom([[2500.0, 2500.0, 50.0]], [[[0.0, 0.0, 50.0]]])
    full = tpx.workspace_bytes(tpx.CALL_GRADIENT_FULL, grid, geom)
    probed = tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=32))
    assert full > 288e9
    # the ring is capped at six times the 6.2 GB of accumulators (a 112-level
    # block, 34 GB): the probed workspace stays under 45 GB, a sixth of the GPU
    assert probed < 45e9
    hist = 401 * 401 * 301 * 2001 * 4.0   # the N x n_t history of Eq. 3
    assert hist / probed > 8.5


def test_probe_side_validated():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])
    ok = tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=4, dtt_side=1))
    assert ok == tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=4))
    with pytest.raises(tpx.TpxError):
        tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=4, dtt_side=2))


def test_range_finder_probe_validation_and_workspace():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0]] * 2, [[[10.0 * i, 0, 20.0] for i in range(6)]] * 2)
    p = tpx.Probe(kind="range_finder", r=4, seed=3)
    # FP64 scratch: D^T Z (S*nrec*r), D D^T Z (S*nt*r), and the tall-skinny QR's
    # segment partials (S*16*nrec*16), reflector coefficients and stacked R
    # factors of P = 5 panels (S*P*r, S*P*r*r) and Q rows (S*nt*r); each region
    # 256-byte aligned
    need = tpx.workspace_bytes(tpx.CALL_RANGE_FINDER, grid, geom, p)
    doubles = 2 * 6 * 4 + 2 * 100 * 4 + (2 * 16 * 6 * 16 + 2 * 5 * 4 + 2 * 5 * 16 + 2 * 100 * 4)
    assert 8 * doubles <= need < 8 * doubles + 3 * 256
    # gradient calls take the kind; r is bounded by nrec and 64
    assert tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, p) > \
        tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=4))
    for bad in (tpx.Probe(kind="range_finder", r=7), tpx.Probe(kind="range_finder", r=65)):
        with pytest.raises(tpx.TpxError):
            tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, bad)
    # the split pair has no observed data
    with pytest.raises(tpx.TpxError):
        tpx.workspace_bytes(tpx.CALL_FORWARD_PROBED, grid, geom, p)
    with pytest.raises(tpx.TpxError):
        tpx.workspace_bytes(tpx.CALL_RANGE_FINDER, grid, geom, tpx.Probe(r=4))


def test_gradient_imaging_condition_needs_vbar():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])
    tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=4, imaging=1, keep_vbar=True))
    for bad in (tpx.Probe(r=4, imaging=1), tpx.Probe(r=4, imaging=2, keep_vbar=True)):
        with pytest.raises(tpx.TpxError):
            tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, bad)


def test_objective_workspace_and_null_arguments():
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0], [200.0, 0, 50.0]], [[[10.0, 0, 20.0]] * 3] * 2)
    fwd = tpx.workspace_bytes(tpx.CALL_FORWARD, grid, geom)
    obj = tpx.workspace_bytes(tpx.CALL_OBJECTIVE, grid, geom)
    # forward ring plus the traces and residuals (2 x S*nt*nrec floats)
    assert obj >= fwd + 2 * 4 * 2 * 100 * 3
    L = tpx.lib()
    g, ge = grid.c(), geom.c()
    ge.wavelet = 0x1000
    # J must not be NULL; nothing is launched
    assert L.tpx_objective(ctypes.byref(g), ctypes.byref(ge), 0x1000, 0x2000, None, None, 0x3000, obj,
                           None) == tpx.E_INVAL


def test_memory_follows_the_papers_estimates():
    # Memory estimates section, Table 1: probing keeps r x N values per pass
    # (u-bar in the forward pass, v-bar in the backward pass, 2 r N in all),
    # where the stored-history gradient keeps N x n_t
    grid = tpx.Grid(**GRID)                       # N = 30 x 40, n_t = 100, 5 padding nodes
    geom = _geom([[100.0, 0, 50.0], [200.0, 0, 50.0]], [[[10.0, 0, 20.0]] * 3] * 2)
    S, N, N_pad, nt = 2, 30 * 40, 40 * 50, 100

    def a(b):
        return (b + 255) // 256 * 256

    for r in (4, 8, 16):
        # u-bar, then a 256-byte header naming the forward pass that wrote it
        assert tpx.state_bytes(grid, geom, tpx.Probe(r=r)) == a(S * r * N * 4) + 256
        keep = tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=r, keep_vbar=True))
        fold = tpx.workspace_bytes(tpx.CALL_GRADIENT_PROBED, grid, geom, tpx.Probe(r=r))
        # v-bar replaces the folded path's one-field partial gradient
        assert keep - fold == a(S * r * N * 4) - a(S * N * 4)
    full = tpx.workspace_bytes(tpx.CALL_GRADIENT_FULL, grid, geom)
    fwd = tpx.workspace_bytes(tpx.CALL_FORWARD, grid, geom)
    assert full - fwd >= (nt - 4) * S * N_pad * 4    # the history: n_t padded fields per shot


def test_largest_shot_field_accepted_and_the_next_rejected():
    # the step kernels address one shot's padded field with 32-bit byte
    # offsets: fields of 2^30 floats or more are refused on the host
    geom = _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])
    ok = tpx.Grid((31_990, 32_000), h=10.0, dt=1.5, nt=10, order=8, nbl=20, damp_vmax=3.0)
    # padded rows of 32,040 + 32 + 4 floats (pitch 32,096) by 32,030 + 8 rows
    assert tpx.workspace_bytes(tpx.CALL_FORWARD, ok, geom) >= 4 * 32_096 * 32_038 * 4
    big = tpx.Grid((33_000, 33_000), h=10.0, dt=1.5, nt=10, order=8, nbl=20, damp_vmax=3.0)
    with pytest.raises(tpx.TpxError) as e:
        tpx.workspace_bytes(tpx.CALL_FORWARD, big, geom)
    assert "2^30" in str(e.value)
    # 3D: 900^3 physical nodes fit (992 x 948 x 948 floats padded), 1000^3 do not
    g3 = dict(h=10.0, dt=1.0, nt=10, order=8, nbl=20, damp_vmax=3.0)
    geom3 = _geom([[100.0, 100.0, 50.0]], [[[10.0, 10.0, 20.0]]])
    assert tpx.workspace_bytes(tpx.CALL_FORWARD, tpx.Grid((900, 900, 900), **g3), geom3) >= 3 * 992 * 948 * 948 * 4
    with pytest.raises(tpx.TpxError):
        tpx.workspace_bytes(tpx.CALL_FORWARD, tpx.Grid((1000, 1000, 1000), **g3), geom3)


def test_binding_checks_tensors_before_any_call():
    # host tensors, wrong dtypes and wrong shapes are refused by the binding
    import torch
    grid = tpx.Grid(**GRID)
    geom = _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]]])
    m_cpu = torch.ones(30, 40)
    with pytest.raises(TypeError):
        tpx.forward(grid, geom, m_cpu)
    with pytest.raises(TypeError):
        tpx.gradient_probed(grid, geom, tpx.Probe(r=4), m_cpu, torch.zeros(1, 100, 1))
    with pytest.raises(TypeError):
        tpx.gradient_full(grid, geom, torch.ones(30, 40, dtype=torch.float64), torch.zeros(1, 100, 1))


def test_table_sizes_do_not_depend_on_earlier_calls():
    # The host image of the injection tables reuses its storage between calls on
    # a thread.  Workspace sizes (which include the tables) must depend on the
    # problem only: a large receiver spread (megabytes of dense maps) and a small
    # one, queried in either order and under both 2D launch depths, give the
    # same answers every time.
    from paper_2104_00794_amd.inputs import workload
    wl = workload("c1_layered_2d_16shots")
    big_g = tpx.Grid(wl.shape, h=wl.h, dt=wl.dt, nt=wl.nt, order=wl.order, nbl=wl.nbl, damp_vmax=wl.vmax)
    big = (big_g, tpx.Geometry(wl.src_pos(), wl.rec_pos()), tpx.Probe(r=16))
    small = (tpx.Grid(**GRID), _geom([[100.0, 0, 50.0]], [[[10.0, 0, 20.0]] * 3]), tpx.Probe(r=8))
    calls = (tpx.CALL_FORWARD, tpx.CALL_GRADIENT_PROBED)
    old = tpx.get_option(tpx.OPT_STEPS_2D)
    try:
        seen = {}
        for steps in (3, 2, 3, 2):
            tpx.set_option(tpx.OPT_STEPS_2D, steps)
            for name, (g, geo, p) in (("big", big), ("small", small), ("big", big), ("small", small)):
                for call in calls:
                    n = tpx.workspace_bytes(call, g, geo, p)
                    assert n > 0
                    assert seen.setdefault((steps, name, call), n) == n, (steps, name, call)
        # the three-step layout adds its own tables (and two plain-pass slots)
        assert seen[(3, "big", tpx.CALL_GRADIENT_PROBED)] > seen[(2, "big", tpx.CALL_GRADIENT_PROBED)]
    finally:
        tpx.set_option(tpx.OPT_STEPS_2D, old)
