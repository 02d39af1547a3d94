"""Shared helpers for the GPU parity tests (no arithmetic of the method here)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def tucker_to_full(core, factors):
    from oracle import tensor
    return tensor.tucker_full(core, factors)


def log(*args):
    print(*args, flush=True)
