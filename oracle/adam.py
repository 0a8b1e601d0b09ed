"""Oracle: one Adam step (Kingma and Ba, 2015), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Used to check the
refinement of the CP factors, which is not part of the paper.
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """Returns (p, m, v) after step number ``step`` (1-based)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
