"""CPU tests of the serving layer's admission policy (host logic only)."""
from paper_2104_00794_amd.serve import admission_plan


def _plan(reqs, slots=4, free=100.0, budget=100.0, nlarge=0, max_large=2):
    size = dict(reqs)
    return admission_plan([k for k, _ in reqs], slots, free, budget, nlarge, max_large,
                          lambda k: size[k], lambda k: k.startswith("L"))


def test_arrival_order_up_to_the_free_slots():
    admit, reject = _plan([("a", 10), ("b", 10), ("c", 10), ("d", 10), ("e", 10)], slots=3)
    assert admit == ["a", "b", "c"] and reject == []


def test_larger_than_the_budget_is_rejected_and_the_scan_goes_on():
    admit, reject = _plan([("a", 150), ("b", 10)])
    assert reject == ["a"] and admit == ["b"]


def test_memory_is_granted_in_arrival_order():
    # b does not fit the free bytes: c, which would, waits behind it
    admit, reject = _plan([("a", 50), ("b", 60), ("c", 10)], free=100.0)
    assert admit == ["a"] and reject == []


def test_a_blocked_large_request_lets_smaller_ones_pass():
    admit, _ = _plan([("L1", 10), ("s1", 10), ("L2", 10), ("s2", 10)], nlarge=2, max_large=2)
    assert admit == ["s1", "s2"]
    admit, _ = _plan([("L1", 10), ("s1", 10), ("L2", 10), ("L3", 10)], nlarge=1, max_large=2)
    assert admit == ["L1", "s1"]   # one more large job fits beside the running one


def test_no_slots_admits_nothing():
    assert _plan([("a", 1)], slots=0) == ([], [])


# --------------------------------------------------------------------------- #
# the workspace arena (first fit, coalescing frees)
# --------------------------------------------------------------------------- #

def _arena(n):
    from paper_2104_00794_amd.serve import Arena
    return Arena(n, device="cpu")


def test_arena_first_fit_alignment_and_views():
    a = _arena(10 * 4096)
    o1, v1 = a.alloc(100)
    o2, v2 = a.alloc(5000)          # two pages
    assert (o1, o2) == (0, 4096) and v1.numel() == 100 and v2.numel() == 5000
    assert v2.data_ptr() - a.buf.data_ptr() == 4096
    assert a.free == [(3 * 4096, 7 * 4096)]
    assert a.alloc(8 * 4096) is None    # larger than what is left
    o3, _ = a.alloc(7 * 4096)
    assert o3 == 3 * 4096 and a.free == []


def test_arena_release_merges_neighbours_and_first_fit_reuses_holes():
    a = _arena(8 * 4096)
    blocks = [a.alloc(4096)[0] for _ in range(8)]
    assert a.free == []
    a.release(blocks[2], 4096)
    a.release(blocks[4], 4096)
    a.release(blocks[3], 4096)          # joins both neighbours: one hole of three pages
    assert a.free == [(2 * 4096, 3 * 4096)]
    assert a.alloc(4 * 4096) is None    # fragmented: 3 pages here, none elsewhere
    o, _ = a.alloc(2 * 4096)
    assert o == 2 * 4096 and a.free == [(4 * 4096, 4096)]
    for b in (0, 1, 5, 6, 7):
        a.release(blocks[b], 4096)
    a.release(2 * 4096, 2 * 4096)
    assert a.free == [(0, 8 * 4096)] and a.free_bytes() == 8 * 4096


def test_arena_refuses_a_double_release():
    import pytest
    a = _arena(4 * 4096)
    o, _ = a.alloc(4096)
    a.release(o, 4096)
    with pytest.raises(ValueError):
        a.release(o, 4096)
