"""Writes tests/golden/cfg3_restricted_s64.npy: the exact control of the n=2047 configuration
(3D, alpha=1/2, beta=1, gamma=1e-2, rank-8 right-hand side of workloads.cfg3) on the sub-grid
i = 64 p - 1 (p = 1..31, 0-based indices), computed by oracle.exact only.

    python tests/golden/make_cfg3_oracle.py [workers]
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import exact  # noqa: E402

STRIDE = 64
OUT = os.path.join(HERE, "cfg3_restricted_s64.npy")


def _part(args):
    slabs, = args
    p = workloads.cfg3()
    rows = [workloads.restriction_rows(p.n, STRIDE)] * 3
    return exact.solve_cp_restricted_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, rows, slabs)


def main(workers):
    p = workloads.cfg3()
    chunks = [list(range(i, p.n, workers * 4)) for i in range(workers * 4)]
    t0 = time.time()
    with ProcessPoolExecutor(workers) as ex:
        parts = list(ex.map(_part, [(c,) for c in chunks]))
    u = np.sum(parts, axis=0)
    np.save(OUT, u)
    print("wrote %s shape %s in %.1fs" % (OUT, u.shape, time.time() - t0))


if __name__ == "__main__":
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
