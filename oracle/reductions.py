"""Per-level horizontal reductions of the projection's outputs.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product
path imports this module.

The paper's I/O server turns prognostic fields into diagnostics with generic
actions, among them reductions of a field over the horizontal (Sec. 3, the
I/O server paragraphs). This is that diagnostic for the projection's outputs,
by its definition: for each field and level, the mean and the maximum over
the nx*ny points of the level.
"""
from __future__ import annotations

import numpy as np


def level_stats(u, v, w, p):
    """Array (4, 2, nz): [field u, v, w, p][mean, max][level k], in FP64."""
    out = []
    for f in (u, v, w, p):
        f = np.asarray(f, dtype=np.float64)
        out.append([f.mean(axis=(1, 2)), f.max(axis=(1, 2))])
    return np.asarray(out)
