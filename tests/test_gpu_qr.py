"""The gauge factorisation of the TDVP sweep on the device (shifted
CholeskyQR in three passes) through the C ABI, against the definition of a QR
(LQ) factorisation: Q has orthonormal columns (rows), the product reproduces
M, the triangular factor has a real positive diagonal, and for well-
conditioned M it equals LAPACK's factor in the same gauge.  Sizes cover the
register Cholesky kernel (n <= 128: one column per lane up to n = 64, two
above, rows dealt unevenly over the wavefronts), the LDS kernel (n = 140) and
the global-memory path (n = 200); condition numbers up to 1e10, as the
Schmidt spectra kept at a 1e-10 cutoff produce."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def graded(rows, cols, cond, rng):
    k = min(rows, cols)
    U, _ = np.linalg.qr(rng.standard_normal((rows, k)) + 1j * rng.standard_normal((rows, k)))
    V, _ = np.linalg.qr(rng.standard_normal((cols, k)) + 1j * rng.standard_normal((cols, k)))
    s = np.logspace(0, -np.log10(cond), k)
    return (U * s) @ V.conj().T


def positive_gauge(R):
    ph = np.diag(R) / np.abs(np.diag(R))
    return R * ph.conj()[:, None]


CASES = [(700, 1, 1.0), (12, 5, 1.0), (40, 16, 1e4), (4000, 65, 1e8), (300, 17, 1e8),
         (500, 23, 1.0), (1000, 64, 1e10),
         (2000, 100, 1e6), (12800, 128, 1e10), (3000, 127, 1e3), (1500, 140, 1e6),
         (2000, 200, 1e4)]


@pytest.mark.parametrize("rows,cols,cond", CASES)
def test_qr(ctx, rows, cols, cond):
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(rows + cols)
    M = graded(rows, cols, cond, rng)
    Q, R = api.qr(ctx, M)
    orth = np.abs(Q.conj().T @ Q - np.eye(cols)).max()
    back = np.linalg.norm(Q @ R - M) / np.linalg.norm(M)
    say(f"[qr] {rows}x{cols} cond {cond:.0e}: |Q^H Q - I| {orth:.1e}, |QR - M|/|M| {back:.1e}")
    assert orth < 1e-13
    assert back < 1e-14
    assert np.abs(np.tril(R, -1)).max() == 0.0
    d = np.diag(R)
    assert np.all(d.real > 0) and np.all(d.imag == 0)
    if cond <= 1e4:
        Rn = positive_gauge(np.linalg.qr(M, mode="r"))
        err = np.abs(R - Rn).max() / np.abs(Rn).max()
        say(f"[qr]   R vs LAPACK {err:.1e}")
        assert err < 1e-12 * cond


@pytest.mark.parametrize("rows,cols,cond", [(5, 12, 1.0), (16, 64, 1e6), (128, 12800, 1e10),
                                            (65, 900, 1e2)])
def test_lq(ctx, rows, cols, cond):
    from paper_2003_13245_amd import api
    rng = np.random.default_rng(7 * rows + cols)
    M = graded(rows, cols, cond, rng)
    L, Q = api.qr(ctx, M, lq=True)
    orth = np.abs(Q @ Q.conj().T - np.eye(rows)).max()
    back = np.linalg.norm(L @ Q - M) / np.linalg.norm(M)
    say(f"[lq] {rows}x{cols} cond {cond:.0e}: |Q Q^H - I| {orth:.1e}, |LQ - M|/|M| {back:.1e}")
    assert orth < 1e-13
    assert back < 1e-14
    assert np.abs(np.triu(L, 1)).max() == 0.0
    d = np.diag(L)
    assert np.all(d.real > 0) and np.all(d.imag == 0)


def test_qr_rejects_bad_shapes(ctx):
    from paper_2003_13245_amd import api
    with pytest.raises(api.FtdError):
        api.qr(ctx, np.ones((3, 5)))
    with pytest.raises(api.FtdError):
        api.qr(ctx, np.ones((5, 3)), lq=True)
