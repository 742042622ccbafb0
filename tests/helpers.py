"""Error metrics and small utilities shared by the tests and the bench.

None of this is projection arithmetic: the metrics compare two results."""
import numpy as np


def relerr(x, ref):
    """Normwise max relative error max|x - ref| / max|ref| (0 if ref == 0).

    Complex arrays keep their dtype, so the modulus of the complex
    difference (real and imaginary parts together) is what is measured."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    if x.shape != ref.shape:
        raise ValueError(f"shape mismatch {x.shape} vs {ref.shape}")
    if np.iscomplexobj(x) != np.iscomplexobj(ref):
        raise TypeError("relerr compares real with real and complex with complex")
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    diff = float(np.max(np.abs(x - ref))) if ref.size else 0.0
    return diff / scale if scale > 0 else diff


def max_field_relerr(out, ref):
    """Max over p, u, v, w of relerr (the headline error of one projection)."""
    return max(relerr(out[k], ref[k]) for k in ("u", "v", "w", "p"))
