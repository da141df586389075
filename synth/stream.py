"""Seeded request arrivals for the streaming workload (input generation only)."""
from __future__ import annotations

import numpy as np


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds, float64, ascending, first at 0) of n requests of a
    Poisson process with `rate` requests per second: exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)
