"""Error metrics and small utilities shared by the tests and the bench.

None of this is projection arithmetic: the metrics compare two results."""
import numpy as np


def relerr(x, ref):
    """Normwise max relative error max|x - ref| / max|ref| (0 if ref == 0)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    diff = np.max(np.abs(x - ref)) if ref.size else 0.0
    return float(diff / scale) if scale > 0 else float(diff)


def max_field_relerr(out, ref):
    """Max over p, u, v, w of relerr (the headline error of one projection)."""
    return max(relerr(out[k], ref[k]) for k in ("u", "v", "w", "p"))
