"""GPU parity of the complex split-plane GEMM kernel against numpy on seeded
operands: every transpose/conjugate combination, ragged tails, split-K."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (16, 16, 4), (64, 64, 16), (37, 53, 29), (5, 130, 3), (128, 128, 4000),
          (200, 70, 1)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (0, 2), (1, 0), (2, 0), (2, 2)])
def test_gemm_f64(ctx, shape, ta, tb):
    from paper_2003_13245_amd import api
    M, N, K = shape
    print(f"[gemm] f64 shape={shape} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    A = cplx(M, K) if ta == 0 else cplx(K, M)
    B = cplx(K, N) if tb == 0 else cplx(N, K)
    opA = A if ta == 0 else (A.T if ta == 1 else A.conj().T)
    opB = B if tb == 0 else (B.T if tb == 1 else B.conj().T)
    ref = opA @ opB
    got = api.gemm(ctx, A, B, ta, tb, "c128")
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    assert err < 1e-13 * max(1, K) ** 0.5, err


@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_f32(ctx, shape):
    from paper_2003_13245_amd import api
    M, N, K = shape
    print(f"[gemm] f32 shape={shape}", flush=True)
    rng = np.random.default_rng(7 + M + N + K)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    ref = A32 @ B32
    got = api.gemm(ctx, A, B, 0, 0, "c64")
    err = np.abs(got - ref).max() / (np.abs(A32).max() * np.abs(B32).max() * K)
    assert err < 2e-6, err


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (2, 0), (2, 2)])
def test_gemm_bf16x3(ctx, shape, ta, tb):
    """bf16 matrix cores with split operands (hi + lo, three products per real
    product): the float32-rounded inputs' product to a relative error of
    order 2^-17 per term."""
    from paper_2003_13245_amd import api
    M, N, K = shape
    print(f"[gemm] bf16x3 shape={shape} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(11 + M + 3 * N + 7 * K)
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    A = cplx(M, K) if ta == 0 else cplx(K, M)
    B = cplx(K, N) if tb == 0 else cplx(N, K)
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    opA = A32 if ta == 0 else (A32.T if ta == 1 else A32.conj().T)
    opB = B32 if tb == 0 else (B32.T if tb == 1 else B32.conj().T)
    ref = opA @ opB
    got = api.gemm(ctx, A, B, ta, tb, "bf16x3")
    scale = np.abs(A32).max() * np.abs(B32).max()
    err = np.abs(got - ref).max() / (scale * max(1, K) ** 0.5)
    assert err < 1e-4, err
    # and clearly better than a single bf16 product (relative ~2^-9)
    assert np.abs(got - ref).max() < 1e-3 * scale * K
