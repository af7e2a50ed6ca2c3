"""Helpers shared by the GPU tests."""
import numpy as np


def rel_fro(got, ref) -> float:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (d if d > 0 else 1.0))
