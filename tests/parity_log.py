"""Normwise comparison helper for the GPU parity tests: prints the difference it achieved
next to its bound, then asserts it (so the margin of every R comparison is in the log)."""
import inspect

import numpy as np


def assert_rel(A, B, bound, what="R"):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = np.linalg.norm(B)
    rd = float(np.linalg.norm(A - B) / (nb if nb > 0 else 1.0))
    caller = inspect.stack()[1].function
    print(f"[parity] {caller}: {what} rel diff {rd:.3e} (bound {bound:.1e}, margin {bound / max(rd, 1e-300):.1e}x)")
    assert rd <= bound, (what, rd, bound)
    return rd
