"""Helpers shared by the GPU tests (no filtering arithmetic here)."""
import numpy as np


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


def max_over_peak(y, ref):
    """The paper's accuracy metric: max |error| / max |reference| (Sec. IV-F)."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(ref)), 1e-300))


def tol_for(K):
    """rel-L2 bound: 1e-5 up to order 8 (K <= 4), 1e-4 at order 16 (K = 8)."""
    return 1e-5 if K <= 4 else 1e-4
