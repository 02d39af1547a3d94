"""tp_inner_noalloc (the inner product with its temporaries in the library's fixed device scratch,
result left in device memory) against tp_inner, which takes them from the context's workspace: the
same kernels on the same inputs, so the two agree to rounding (bitwise when the contractions split
alike).  Two calls in a row, the second on smaller tensors, in FP64 and in mixed precision, 3D and
2D; the empty case; and a pair whose temporaries exceed the scratch is rejected before any work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _tucker(tp, d, ns, ranks, cap, prec, seed):
    """A Tucker tensor with the given ranks and seeded N(0,1) core and factors (the inner product
    needs no orthonormality)."""
    import torch
    X = tp.Tensor(d, ns, cap, prec)
    rng = np.random.default_rng(seed)
    dt = torch.float64 if prec == 0 else torch.float32
    core = rng.standard_normal(int(np.prod(ranks)))
    X.core[: core.size] = torch.as_tensor(core, dtype=dt, device="cuda")
    for m in range(d):
        f = rng.standard_normal(ns[m] * ranks[m])
        X.factors[m][: f.size] = torch.as_tensor(f, dtype=dt, device="cuda")
        X.s.rank[m] = ranks[m]
    X._sync_ranks()
    return X


def _numpy_inner(X, Y):
    """<X, Y> from the host copies: sum over the cores of Cx x_l (Vx^T Vy) with Cy."""
    cx, fx = X.numpy_parts()
    cy, fy = Y.numpy_parts()
    G = [a.T @ b for a, b in zip(fx, fy)]
    if len(G) == 3:
        return float(np.einsum("abc,ai,bj,ck,ijk->", cx, G[0], G[1], G[2], cy))
    return float(np.einsum("ab,ai,bj,ij->", cx, G[0], G[1], cy))


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


CASES = [
    # (d, grid sizes, ranks of x, ranks of y, cap, prec): each pair of consecutive cases is one call
    # followed by a smaller one
    (3, (255, 255, 255), (40, 36, 44), (48, 30, 40), 64, 0),
    (3, (127, 63, 31), (10, 12, 5), (7, 9, 11), 64, 0),
    (3, (2047, 2047, 2047), (56, 50, 52), (50, 56, 49), 64, 1),
    (3, (511, 255, 127), (20, 8, 16), (12, 17, 3), 64, 1),
    (2, (1023, 511), (60, 40), (33, 47), 64, 0),
    (2, (63, 31), (5, 9), (12, 3), 64, 1),
]


@pytest.mark.parametrize("pair", [0, 1, 2])
def test_noalloc_inner_matches_workspace_inner(ctx, pair):
    import paper_1809_01971_amd as tp
    import torch
    for case in CASES[2 * pair: 2 * pair + 2]:
        d, ns, rx, ry, cap, prec = case
        print("noalloc inner: d=%d n=%s ranks %s x %s prec=%d" % (d, ns, rx, ry, prec), flush=True)
        X = _tucker(tp, d, ns, rx, cap, prec, seed=11)
        Y = _tucker(tp, d, ns, ry, cap, prec, seed=12)
        ref = ctx.inner(X, Y)
        out = ctx.inner_noalloc(X, Y)
        got = float(out.cpu()[0])
        host = _numpy_inner(X, Y)
        print("  tp_inner %.17g  noalloc %.17g  numpy %.17g" % (ref, got, host), flush=True)
        # same kernels, same contraction splits: identical up to the last bits
        assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-300)
        # and both are the inner product of the tensors the host holds (FP64 sums of the stored values)
        scale = np.sqrt(ctx.inner(X, X) * ctx.inner(Y, Y))
        assert abs(got - host) <= 1e-12 * scale
        torch.cuda.synchronize()


def test_noalloc_inner_empty_and_oversized(ctx):
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import TP_EINVAL, TPError
    X = _tucker(tp, 3, (63, 63, 63), (4, 5, 6), 8, 0, seed=1)
    Z = tp.Tensor(3, 63, 8, 0)          # ranks 0: the zero tensor
    out = ctx.inner_noalloc(X, Z)
    assert float(out.cpu()[0]) == 0.0
    # ranks 128 x 128 x 128: three dense FP64 cores of 16 MiB each do not fit the 16 MiB scratch
    A = _tucker(tp, 3, (255, 255, 255), (128, 128, 128), 128, 0, seed=2)
    with pytest.raises(TPError) as e:
        ctx.inner_noalloc(A, A)
    assert e.value.status == TP_EINVAL
    # the entry point still works after the rejection
    B = _tucker(tp, 3, (63, 63, 63), (6, 5, 4), 8, 0, seed=3)
    assert abs(float(ctx.inner_noalloc(X, B).cpu()[0]) - ctx.inner(X, B)) <= 1e-13 * abs(ctx.inner(X, B))
