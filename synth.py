"""Seeded synthetic inputs shared by the tests and the benchmark.

Only random numbers and bookkeeping live here: none of the method's
arithmetic.  Initial turbulent fields are drawn by the method itself
(init_field, on both the oracle and the GPU side, from seeds).
"""

import numpy as np


def normal_field(shape, seed, scale=1.0):
    """float64 array of independent N(0, scale^2) values."""
    return scale * np.random.default_rng(seed).standard_normal(shape)


def evenly_spaced_steps(n_steps, n_times):
    """n_times step indices evenly spaced over [0, n_steps] including both ends."""
    if n_times == 1:
        return [n_steps]
    return sorted({int(round(i * n_steps / (n_times - 1))) for i in range(n_times)})


def every_k_steps(n_steps, k):
    return list(range(0, n_steps + 1, k))
