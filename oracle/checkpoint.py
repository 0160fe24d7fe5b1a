"""Cost of reversing a time-stepping chain under a snapshot budget (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The gradient runs the adjoint steps in reverse order, each needing the forward
state at its start (Sec. I and Sec. II.A: the adjoint is integrated backward
along the stored forward trajectory, with checkpointing).  With room for only
a few states, forward steps are recomputed from the stored ones.  The unit of
work here is one "step" of the chain; the library applies it to segments of
several time steps.

Reversal of l steps, starting with the state at the first step held and s
further snapshot slots free: reversing the last remaining step costs no
advance (its store-mode evaluation is not counted); with no free slot, step i
is reached by advancing i steps from the held state; otherwise the cheapest
plan advances m steps, stores that state, reverses the last l - m steps with
one slot fewer and then the first m steps with the slot freed again, for the
best m.  This recursive structure is that of the optimal binomial schedules
(Griewank, 1992; Griewank & Walther, 2000); min_advances evaluates it by plain
dynamic programming over every split, the slow definition of the optimum.
"""

from functools import lru_cache


@lru_cache(maxsize=None)
def _cost(n, k):
    if n == 1:
        return 0
    if k == 0:
        # step i (0-based) is reached by advancing i steps from the held state
        return sum(range(n))
    return min(m + _cost(n - m, k - 1) + _cost(m, k) for m in range(1, n))


def min_advances(l, s):
    """Fewest single-step advances that reverse l >= 1 steps with the first
    state held and s >= 0 free snapshot slots."""
    if l < 1 or s < 0:
        raise ValueError("need l >= 1 and s >= 0")
    # fill the table bottom-up so the recursion stays shallow
    for n in range(1, l + 1):
        for k in range(0, s + 1):
            _cost(n, k)
    return _cost(l, s)


def optimal_first_advances(l, s):
    """Every first advance m (1 <= m < l) that attains min_advances(l, s), s >= 1."""
    if l < 2 or s < 1:
        raise ValueError("need l >= 2 and s >= 1")
    best = min_advances(l, s)
    return [m for m in range(1, l) if m + min_advances(l - m, s - 1) + min_advances(m, s) == best]
