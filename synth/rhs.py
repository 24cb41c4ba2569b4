"""Seeded random stage data (input vectors only): right-hand sides, Dirichlet trace values,
initial states.  Stream 4 of the workload's seed sequence, sub-keyed by ``key``."""
from __future__ import annotations

import numpy as np


def random_vector(n: int, cfg_id: int, key: int = 0, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg_id), 4, int(key)]))
    return scale * rng.standard_normal(int(n))
