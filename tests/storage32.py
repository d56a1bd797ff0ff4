"""Model of FP32 population storage for the oracle (test-side).

The library keeps populations in HBM as deviations from a constant, direction-symmetric reference
(f_i - w_i; g_i; k_0 - 1/3 and k_i for i > 0) and rounds each deviation to FP32 once per step, when the
post-collision state is stored.  Propagation and half-way bounce-back only permute values between
directions of equal reference, so rounding the post-propagation state s_{t+1} of an FP64 oracle step in
the same representation gives the state an FP32-storage run would hold, up to the rounding of its own
FP64 arithmetic.  An oracle run with this rounding after every step (and of the initial state) measures
the error that FP32 storage alone brings, independently of the GPU.
"""
from __future__ import annotations

import numpy as np


def reference(lattice):
    """[species][Q] reference values: f: w_i; g: 0; k: 1/3 at i = 0."""
    if lattice == 0:
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    else:
        w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    r = np.zeros((3, w.size))
    r[0] = w
    r[2, 0] = 1.0 / 3.0
    return r


def round_state(pop, lattice):
    """pop [3][Q][N] (FP64, in place): each population rounded to FP32 relative to its reference."""
    r = reference(lattice)[:, :, None]
    pop -= r
    pop[...] = pop.astype(np.float32).astype(np.float64)
    pop += r
    return pop


def run_fp32_storage(orc, p, pop, steps, h=None):
    """Oracle steps with the state rounded as FP32 storage would round it after each step."""
    round_state(pop, p.lattice)
    for _ in range(steps):
        orc.step(p, pop, 1, h)
        round_state(pop, p.lattice)
    return pop
