"""Host-side binomial checkpoint schedule of the library (no device needed).

The schedule reverses L segments with a budget of snapshot slots.  A small
interpreter replays it: every advance starts from a slot holding its first
boundary (or from the state the previous advance left), every reverse comes
in the order L-1, ..., 0 from a slot or live state at its boundary, slot 0
keeps boundary 0, no slot index leaves the budget, and the advances before
the first reverse form one chain from boundary 0 (the forward sweep).  Its
advance count must equal the oracle's fewest advances for that budget.
"""

import ctypes

import pytest

import oracle as O

ADVANCE, REVERSE = 0, 1


def _lib():
    from paper_2602_14016_amd import native
    import os
    if not os.path.exists(native.LIB_PATH):
        from paper_2602_14016_amd import build
        build.build(verbose=False)
    return native.load(), native


def schedule(L, slots):
    lib, native = _lib()
    n = ctypes.c_int64()
    native.check(lib.pa_checkpoint_schedule(L, slots, None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * (5 * max(n.value, 1)))()
    native.check(lib.pa_checkpoint_schedule(L, slots, buf, n.value, ctypes.byref(n)))
    return [tuple(buf[5 * i: 5 * i + 5]) for i in range(n.value)]


def advances(L, slots):
    lib, native = _lib()
    a = ctypes.c_int64()
    native.check(lib.pa_checkpoint_advances(L, slots, ctypes.byref(a)))
    return a.value


def replay(acts, L, slots):
    """Check the schedule's validity; return the number of segment advances."""
    held = {0: 0}            # slot -> boundary
    live = 0                 # boundary of the live state, None if unknown
    next_rev = L - 1
    seen_reverse = False
    n_adv = 0
    for kind, a, b, src, dst in acts:
        if src == -1:
            assert live == a, "start from a live state that is not at the boundary"
        else:
            assert 0 <= src < slots and held.get(src) == a, "start from a slot not holding the boundary"
        if not seen_reverse:
            assert src == -1, "forward sweep must be one chain from boundary 0"
        if kind == ADVANCE:
            assert a < b <= next_rev, "advance past the next segment to reverse"
            n_adv += b - a
            live = b
            if dst != -1:
                assert 1 <= dst < slots, "slot 0 must keep boundary 0"
                held[dst] = b
        else:
            assert kind == REVERSE and b == a + 1 and dst == -1
            assert a == next_rev, "segments must be reversed in order L-1, ..., 0"
            seen_reverse = True
            next_rev -= 1
            live = None
            for s in [s for s, bd in held.items() if bd > a and s != 0]:
                del held[s]   # states past the reversed segment are never needed again
    assert next_rev == -1, "every segment reversed"
    return n_adv


@pytest.mark.parametrize("slots", [1, 2, 3, 4, 5, 7])
def test_schedule_is_valid_and_optimal(slots):
    for L in range(1, 61):
        acts = schedule(L, slots)
        n_adv = replay(acts, L, min(slots, L))
        assert n_adv == advances(L, slots) == O.min_advances(L, slots - 1), (L, slots)


def test_schedule_with_a_slot_per_boundary_is_the_uniform_one():
    # with L slots the schedule advances one segment at a time, keeping each boundary,
    # then reverses from the kept states: the one-checkpoint-per-segment sweep
    L = 9
    acts = schedule(L, L)
    fwd = acts[:L - 1]
    assert [(k, a, b, src) for k, a, b, src, _ in fwd] == [(ADVANCE, i, i + 1, -1) for i in range(L - 1)]
    assert [a for k, a, *_ in acts if k == REVERSE] == list(range(L - 1, -1, -1))
    assert advances(L, L) == advances(L, 100) == L - 1


def test_long_horizon_counts():
    # closed form at sizes the oracle's table does not reach: slots = 2 reverses L
    # segments with t advances each where C(t + 2, 2) >= L
    for L in (1000, 20000, 123457):
        t = 0
        while (t + 1) * (t + 2) // 2 < L:
            t += 1
        import math
        assert advances(L, 2) == t * L - math.comb(t + 2, 3)
    assert advances(100000, 1) == 100000 * 99999 // 2
    n = len(schedule(20000, 40))
    assert n > 20000


def test_schedule_argument_errors():
    lib, native = _lib()
    n = ctypes.c_int64()
    a = ctypes.c_int64()
    assert lib.pa_checkpoint_advances(0, 3, ctypes.byref(a)) != 0
    assert lib.pa_checkpoint_advances(5, 0, ctypes.byref(a)) != 0
    assert lib.pa_checkpoint_schedule(5, 0, None, 0, ctypes.byref(n)) != 0
    buf = (ctypes.c_int32 * 5)()
    assert lib.pa_checkpoint_schedule(6, 2, buf, 1, ctypes.byref(n)) != 0
    assert n.value > 1
    # a schedule is a host list of about two actions per segment: bounded
    assert lib.pa_checkpoint_schedule((1 << 22) + 1, 3, None, 0, ctypes.byref(n)) == -1
    assert b"PA_MAX_SCHEDULE_SEGMENTS" in lib.pa_last_error()
    assert lib.pa_checkpoint_advances((1 << 22) + 1, 3, ctypes.byref(a)) == 0 and a.value > 0
    assert lib.pa_set_checkpoint_slots(None, 3) != 0
