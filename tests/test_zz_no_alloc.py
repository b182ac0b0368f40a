"""ftd_gemm_noalloc, the entry point that allocates nothing, against ftd_gemm
(the same product from host buffers) through the C ABI: bit-identical
results on two calls in a row, the second smaller, in both precisions, and
not a single allocation through the context's allocator during the calls.
Both calls use split-K partial sums, so the second reads the scratch array
the first left behind and must not depend on it."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class _CountingAllocator:
    def __init__(self):
        import torch
        self.torch = torch
        self.count = 0

    def alloc(self, nbytes):
        self.count += 1
        s = self.torch.cuda.current_stream(0).cuda_stream
        return self.torch.cuda.caching_allocator_alloc(nbytes, 0, s)

    def free(self, ptr):
        self.torch.cuda.caching_allocator_delete(ptr)


def _planar(x, dtype):
    import torch
    flat = np.concatenate([x.real.reshape(-1), x.imag.reshape(-1)]).astype(dtype)
    return torch.from_numpy(flat).cuda()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_gemm_noalloc_equals_gemm(precision):
    import torch
    from paper_2003_13245_amd import api
    al = _CountingAllocator()
    ctx = api.Context(0, allocator=al)
    rng = np.random.default_rng(21)
    dt = np.float64 if precision == "c128" else np.float32
    # (M, N, K, transA, transB): split-K in both; the second call is smaller
    for M, N, K, ta, tb in ((128, 128, 4096, 0, 0), (64, 50, 900, 2, 1)):
        say(f"[noalloc] {precision} M={M} N={N} K={K} transA={ta} transB={tb}")
        a_shape = (M, K) if ta == 0 else (K, M)
        b_shape = (K, N) if tb == 0 else (N, K)
        A = rng.standard_normal(a_shape) + 1j * rng.standard_normal(a_shape)
        B = rng.standard_normal(b_shape) + 1j * rng.standard_normal(b_shape)
        ref = api.gemm(ctx, A, B, ta, tb, precision)
        dA, dB = _planar(A, dt), _planar(B, dt)
        dC = torch.full((2 * M * N,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        before = al.count
        api.gemm_noalloc(ctx, dA, dB, dC, M, N, K, ta, tb, precision)
        ctx.synchronize()
        assert al.count == before, "the allocation-free entry point allocated"
        h = dC.cpu().numpy()
        out = (h[: M * N] + 1j * h[M * N:]).reshape(M, N)
        assert np.array_equal(out, ref), float(np.abs(out - ref).max())
        # and the product itself, to the precision's rounding
        exact = (A if ta == 0 else (A.T if ta == 1 else A.conj().T)) @ \
                (B if tb == 0 else (B.T if tb == 1 else B.conj().T))
        tol = 1e-12 if precision == "c128" else 2e-5
        assert np.abs(out - exact).max() <= tol * np.abs(exact).max() * np.sqrt(K / 64)
    with pytest.raises(api.FtdError) as e:
        big = torch.zeros(2 * 2048 * 1024, dtype=torch.float64, device="cuda")
        api.gemm_noalloc(ctx, big[: 2 * 2048], big[: 2 * 1024], big, 2048, 1024, 1, 0, 0,
                         "c128")
    assert e.value.code == 1
    ctx.close()
