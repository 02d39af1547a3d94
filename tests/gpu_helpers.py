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


def _err_part(args):
    from threadpoolctl import threadpool_limits
    from oracle import exact
    (w, F, alpha, cn, cp, core, T, slabs) = args
    # one BLAS thread per worker: the pool already spreads the slabs over the cores
    with threadpool_limits(limits=1):
        return exact.tucker_error_slabs(w, F, alpha, cn, cp, core, T, slabs)


def global_rel_error(p, core, tfactors, workers=None, stride=1):
    """Exact ||X - u|| / ||u|| over the whole grid (Parseval, slab-parallel over host cores);
    stride > 1 sums every stride-th spectral slab only (an unbiased sample of the error)."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    workers = workers or min(12, os.cpu_count() or 1)
    slabs = list(range(0, p.n, stride))
    chunks = [slabs[i::workers] for i in range(workers)]
    args = [(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, core, tfactors, c) for c in chunks]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with ProcessPoolExecutor(workers) as ex:
        parts = list(ex.map(_err_part, args))
    e2 = sum(a for a, _ in parts)
    u2 = sum(b for _, b in parts)
    return float(np.sqrt(e2 / u2))
