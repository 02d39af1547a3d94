"""Gram eigensolvers of the truncation (tp_gram_eig) against numpy's symmetric eigensolver: the
tridiagonal path (Householder reduction, multisection on qd Sturm counts, twisted-factorisation
eigenvectors; eigenpairs below cut * trace dropped) and the Jacobi path (pivoted Cholesky, one-sided
Jacobi), on Gram matrices of cores with decaying singular values (the spectra the HOSVD sees), on
small orders, and on clustered spectra (which the tridiagonal path hands to the Jacobi path)."""
import numpy as np
import pytest

from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


def _grams(K, decays, seed):
    """Gram matrices M M^T of K x (K^2) unfoldings with singular values 10^(-i/decay) (decay 0: all
    equal, a fully clustered spectrum), random orthogonal factors."""
    rng = np.random.default_rng(seed)
    out = []
    for dec in decays:
        U, _ = np.linalg.qr(rng.standard_normal((K, K)))
        sv = 10.0 ** (-np.arange(K) / dec) if dec else np.ones(K)
        W, _ = np.linalg.qr(rng.standard_normal((K * K, K)))
        M = (U * sv) @ W.T
        out.append(M @ M.T)
    return np.stack(out)


def _check(G, w, v, rank, rest, cut, label):
    """Eigenvalues against numpy, orthonormal kept eigenvectors, residuals, and the HOSVD quantity:
    the mass of G outside the kept span equals the exact eigenvalue tail."""
    K = G.shape[0]
    ref = np.linalg.eigvalsh(G)[::-1]
    nrm = ref[0]
    q = rank
    assert 1 <= q <= K
    Vq = v[:, :q]
    orth = np.abs(Vq.T @ Vq - np.eye(q)).max()
    res = np.abs(G @ Vq - Vq * w[:q]).max() / nrm
    ew = np.abs(w[:q] - ref[:q]).max() / nrm
    outside = (np.trace(G) - np.trace(Vq.T @ G @ Vq)) / np.trace(G)
    tail = ref[q:].clip(min=0).sum() / np.trace(G)
    log("  %s K=%d rank %d: eig %.1e orth %.1e resid %.1e outside %.2e tail %.2e rest %.2e" % (
        label, K, q, ew, orth, res, outside, tail, rest / np.trace(G)))
    assert ew < 1e-13 * K
    assert orth < 1e-10
    assert res < 1e-12 * K
    assert abs(outside - tail) < 1e-12 + 1e-6 * tail
    assert np.all(w[q:] == 0) and np.all(v[:, q:] == 0)
    if cut > 0:
        # dropped eigenvalues are those below cut * trace, and rest is their sum
        assert np.all(ref[:q] > cut * np.trace(G) * (1 - 1e-8))
        assert abs(rest - ref[q:].clip(min=0).sum()) <= 1e-12 * np.trace(G)


@pytest.mark.parametrize("cut", [0.0, 2.3e-12])
@pytest.mark.parametrize("K", [64, 56, 28, 17, 3, 2, 1])
def test_gram_eig_decaying_spectra(ctx, K, cut):
    import torch
    G = _grams(K, [2.0, 5.0, 10.0, 20.0], seed=K)
    w, v, ranks, rest = ctx.gram_eig(torch.as_tensor(G, device="cuda"), cut=cut)
    w, v = w.cpu().numpy(), v.cpu().numpy()
    for b in range(G.shape[0]):
        # the binding's v[b] is the column-major K x K matrix: row k of the torch tensor is column k
        _check(G[b], w[b], v[b].T, ranks[b], rest[b], cut, "cut=%g decay #%d" % (cut, b))


def test_gram_eig_clusters_fall_back(ctx):
    """Equal and nearly equal eigenvalues (a fully clustered spectrum, and pairs of singular values
    equal to 1e-12 relative): the tridiagonal path cannot certify its eigenvectors orthogonal there and
    the Jacobi path takes over; the results meet the same checks."""
    import torch
    K = 64
    G = list(_grams(K, [0.0], seed=5))
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((K, K)))
    sv = np.repeat(10.0 ** (-np.arange(K // 2) / 4.0), 2) * (1 + 1e-12 * np.tile([0, 1], K // 2))
    G.append((U * sv ** 2) @ U.T)
    G = np.stack(G)
    w, v, ranks, rest = ctx.gram_eig(torch.as_tensor(G, device="cuda"), cut=2.3e-12)
    w, v = w.cpu().numpy(), v.cpu().numpy()
    for b in range(G.shape[0]):
        _check(G[b], w[b], v[b].T, ranks[b], rest[b], 0.0, "cluster #%d" % b)


def test_gram_eig_rejects_bad_arguments(ctx):
    import torch
    from paper_1809_01971_amd._tp import TP_EINVAL, TPError
    G = torch.as_tensor(_grams(80, [5.0], seed=1), device="cuda")
    with pytest.raises(TPError) as e:
        ctx.gram_eig(G, cut=1e-10)   # tridiagonal path is limited to K <= 64
    assert e.value.status == TP_EINVAL
    with pytest.raises(TPError) as e:
        ctx.gram_eig(G[:, :8, :8].contiguous(), cut=1e-15)   # below the smallest supported cut
    assert e.value.status == TP_EINVAL
