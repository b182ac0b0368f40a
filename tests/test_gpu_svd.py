"""GPU truncated SVD (the compression kernel) against numpy's SVD on seeded
matrices with a graded spectrum: tall, wide, square, rank deficient."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def graded(rng, M, N, rank, decay=0.5):
    r = min(rank, M, N)
    U, _ = np.linalg.qr(rng.standard_normal((M, r)) + 1j * rng.standard_normal((M, r)))
    V, _ = np.linalg.qr(rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r)))
    s = decay ** np.arange(r)
    return (U * s) @ V.conj().T


@pytest.mark.parametrize("M,N,rank,D", [(40, 10, 10, 4), (15, 10, 10, 6), (10, 40, 10, 3),
                                        (64, 24, 9, 12), (7, 7, 7, 7), (300, 40, 40, 16),
                                        (24, 96, 20, 8), (900, 301, 301, 64)])
@pytest.mark.parametrize("s_left", [True, False])
def test_svd_trunc(ctx, M, N, rank, D, s_left):
    from paper_2003_13245_amd import api
    print(f"[svd] M={M} N={N} rank={rank} D={D} s_left={s_left}", flush=True)
    rng = np.random.default_rng(M * 31 + N)
    T = graded(rng, M, N, rank)
    L, R = api.svd_trunc(ctx, T, D, 1e-10, s_left)
    U, s, Vh = np.linalg.svd(T)
    k = min(D, int((s > 1e-10 * s[0]).sum()))
    assert L.shape[1] == k
    ref = (U[:, :k] * s[:k]) @ Vh[:k]
    assert np.abs(L @ R - ref).max() < 1e-12
    if s_left:
        assert np.allclose(R @ R.conj().T, np.eye(k), atol=1e-12)
    else:
        assert np.allclose(L.conj().T @ L, np.eye(k), atol=1e-12)
