"""Adam update (the training algorithms named in the Methods section,
following Kingma and Ba) in FP64.

Reading: the paper quotes only the learning rate of its MoDL default; the
moment decay rates and epsilon are the Adam paper's defaults
(0.9, 0.999, 1e-8), with bias correction, and epsilon added after the square
root.  ``step`` counts from 1.
"""
from __future__ import annotations

import numpy as np


def step(w, g, m, v, t, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
