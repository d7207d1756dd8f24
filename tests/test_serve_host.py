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
