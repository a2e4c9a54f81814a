"""Seeded synthetic inputs (evaluation points, instance parameters) shared by tests and the benchmark.

Holds none of the scheme's arithmetic: only numpy's PCG64 generator and the shapes of the paper's
workloads (Sec. 4: d from 100 to 10^4, x0 = 0 for Allen-Cahn Case 1, Gaussian or uniform points).
"""
import math

import numpy as np


def points(kind, P, d, seed):
    """x0 [P][d] float64: 'zero', 'normal:<std>' (N(0, std^2 I)), 'normal_over_sqrt_d' (N(0, I/d)),
    'uniform' (U[-1, 1]^d)."""
    rng = np.random.default_rng(seed)
    if kind == "zero":
        return np.zeros((P, d))
    if kind.startswith("normal:"):
        return float(kind.split(":")[1]) * rng.standard_normal((P, d))
    if kind == "normal_over_sqrt_d":
        return rng.standard_normal((P, d)) / math.sqrt(d)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, size=(P, d))
    raise ValueError(kind)


def batched_instances(n_inst=64, seed=0xC2):
    """Uneven HJB instances: lam ~ U[0.5, 2], d uniform over {100, 500, 1000, 5000, 10000}, M uniform over
    the multiples of 64 in [512, 8192]."""
    rng = np.random.default_rng(seed)
    dims = np.array([100, 500, 1000, 5000, 10000])
    out = []
    for i in range(n_inst):
        out.append(dict(instance=i, lam=float(rng.uniform(0.5, 2.0)), d=int(rng.choice(dims)),
                        M=int(64 * rng.integers(8, 129))))
    return out
