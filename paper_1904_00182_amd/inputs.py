"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module only draws random numbers (NumPy PCG64 generators, values in element or
request order); it holds none of the solver's arithmetic.  Designs that the
workloads smooth with a cone filter and threshold are smoothed by each side with its
own filter implementation; this module only supplies the raw noise.
"""

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def noise_design(n_elems, seed, centre=0.5, amplitude=0.1):
    """centre + amplitude * U(-1, 1) per element, drawn in element order."""
    return centre + amplitude * rng(seed).uniform(-1.0, 1.0, n_elems)


def uniform_design(n_elems, seed):
    """U(0, 1) per element, drawn in element order (raw noise before smoothing)."""
    return rng(seed).uniform(0.0, 1.0, n_elems)


def random_vector(n, seed, scale=1.0):
    """Standard-normal test vector (apply-parity inputs)."""
    return scale * rng(seed).standard_normal(n)


def choose_elements(n_elems, count, seed):
    """`count` distinct element indices (finite-difference check points)."""
    return np.sort(rng(seed).choice(n_elems, size=count, replace=False))


def request_stream(n_requests, rate, seed, grids, grs, qh_range=(0.5, 2.0)):
    """Poisson arrivals at `rate` per second plus per-request draws.

    Returns a list of dicts with arrival time, grid, Gr, heat-flux magnitude and the
    design seed (1000 + request index).
    """
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        out.append({
            "id": r,
            "arrival": float(t[r]),
            "grid": tuple(grids[int(g.integers(len(grids)))]),
            "gr": float(grs[int(g.integers(len(grs)))]),
            "q_h": float(g.uniform(*qh_range)),
            "design_seed": 1000 + r,
        })
    return out
