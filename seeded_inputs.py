"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws the random
initial data that both the GPU library and the oracle are given.  Arrays
have shape (n_{d-1}, ..., n_0) with x fastest, n_a = N_a - 1 interior nodes.
"""
import numpy as np


def interior_shape(N):
    return tuple(int(n) - 1 for n in reversed(list(N)))


def uniform_field(seed, N, lo=-0.9, hi=0.9):
    """i.i.d. uniform[lo, hi] nodal values in float64 (one value per mesh point)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=interior_shape(N))


def batch_instances(seed, count, sizes=(128, 192, 256, 384, 512), eps=(0.01, 0.05)):
    """Sizes, eps and initial-data seeds of independent batched instances."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(count + 1)
    rng = np.random.default_rng(children[0])
    Ns = rng.choice(np.asarray(sizes), size=count)
    epss = rng.uniform(eps[0], eps[1], size=count)
    seeds = [int(c.generate_state(1)[0]) for c in children[1:]]
    return [(int(n), float(e), s) for n, e, s in zip(Ns, epss, seeds)]
