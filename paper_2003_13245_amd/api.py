"""Python face of libftdmrg.so (include/ftdmrg.h): argument marshalling only.

Names follow the C ABI: mpo_build, thermal_prep, tdvp_step, corr_current,
mobility, plus the kernel-level entry points used by the tests and the
benchmark.  torch supplies the HIP stream and (optionally) the device
allocator; all computation happens in the native library, which must be
built: importing this module raises ImportError otherwise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _abi
from ._abi import FtdError, PRECISION, check, lib

_SHUTDOWN = [False]
_CONTEXTS = weakref.WeakSet()


@atexit.register
def _release_all():
    # Runs before torch's own exit handlers (this module is imported after
    # torch): every live context is synchronised and destroyed together with
    # its handles while the HIP runtime and torch's allocator are still up.
    for ctx in list(_CONTEXTS):
        try:
            ctx.close()
        except Exception:
            pass
    _SHUTDOWN[0] = True


__all__ = ["Context", "Mpo", "Mps", "mpo_build", "thermal_prep", "tdvp_step", "tdvp_step_expand",
           "tdvp_pair",
           "corr_current", "mobility", "mobility_sweep", "mobility_grad", "mobility_autograd",
           "Mobility", "mean_free_path", "fgr_corr", "reduced_density",
           "coherent_length", "qr", "apply_compress", "overlap", "heff_apply", "mps_from_host",
           "mps_load", "gemm", "FtdError"]


class Context:
    """One library context on a HIP device, bound to a HIP stream.

    stream: an integer hipStream_t, or None for torch's current stream on the
    device (torch required), or 0 for the null stream.
    use_torch_allocator: route device allocations through torch's caching
    allocator."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = True,
                 allocator=None):
        """allocator: optional object with alloc(nbytes) -> device address
        (0 on failure) and free(address), used instead of torch's caching
        allocator (e.g. a pool, or a wrapper that counts or limits)."""
        self._alloc = None
        alloc_p = None
        if stream is None or use_torch_allocator:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
        if allocator is not None:
            def _a(nbytes, user):
                try:
                    return int(allocator.alloc(int(nbytes))) or None
                except Exception:
                    return None

            def _f(ptr, user):
                allocator.free(ptr)
        elif use_torch_allocator:
            dev, st = device, int(stream)

            def _a(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
                except Exception:
                    return None

            def _f(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)
        if allocator is not None or use_torch_allocator:
            self._afn = _abi.ALLOC_FN(_a)
            self._ffn = _abi.FREE_FN(_f)
            self._alloc = _abi.Allocator(self._afn, self._ffn, None)
            alloc_p = C.byref(self._alloc)
        self._stream = int(stream)
        self.device = device
        h = C.c_void_p()
        check(lib.ftd_ctx_create(device, C.c_void_p(self._stream), alloc_p, C.byref(h)))
        self.h = h
        self._handles = weakref.WeakSet()
        _CONTEXTS.add(self)

    def _track(self, handle):
        self._handles.add(handle)

    def close(self):
        """Synchronise and release the native context and every handle created
        from it that is still alive (their later use raises).  Called for all
        live contexts at interpreter exit."""
        h = getattr(self, "h", None)
        if not h:
            return
        lib.ftd_ctx_synchronize(h)
        for obj in list(self._handles):
            obj._release()
        lib.ftd_ctx_destroy(h)
        self.h = None
        _CONTEXTS.discard(self)

    def __del__(self):
        try:
            if getattr(self, "h", None) and not _SHUTDOWN[0]:
                lib.ftd_ctx_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def synchronize(self):
        check(lib.ftd_ctx_synchronize(self.h))

    def set_timing(self, on: bool):
        check(lib.ftd_ctx_set_timing(self.h, int(bool(on))))

    def set_verbose(self, level: int):
        check(lib.ftd_ctx_set_verbose(self.h, int(level)))

    def stats_reset(self):
        check(lib.ftd_ctx_stats_reset(self.h))

    def stats(self) -> dict:
        s = _abi.Stats()
        check(lib.ftd_ctx_stats(self.h, C.byref(s)))
        out = {}
        for k, _ in _abi.Stats._fields_:
            v = getattr(s, k)
            out[k] = list(v) if k.startswith("kind_") else v
        return out


class _Handle:
    _destroy = None

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h
        ctx._track(self)

    def _release(self):
        if self.h:
            type(self)._destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.h and not _SHUTDOWN[0]:
                type(self)._destroy(self.h)
                self.h = None
        except Exception:
            pass


class Mpo(_Handle):
    _destroy = staticmethod(lib.ftd_mpo_destroy)

    def info(self):
        n = C.c_int32()
        check(lib.ftd_mpo_info(self.h, C.byref(n), None, None))
        dims = np.zeros(n.value, dtype=np.int32)
        w = np.zeros(max(1, n.value - 1), dtype=np.int32)
        check(lib.ftd_mpo_info(self.h, C.byref(n), dims.ctypes.data_as(_abi.I32P),
                               w.ctypes.data_as(_abi.I32P)))
        return dims, w[: n.value - 1]


class Mps(_Handle):
    _destroy = staticmethod(lib.ftd_mps_destroy)

    def info(self):
        n = C.c_int32()
        check(lib.ftd_mps_info(self.h, C.byref(n), None, None, None))
        bd = np.zeros(max(1, n.value - 1), dtype=np.int32)
        ln = C.c_double()
        pr = C.c_int32()
        check(lib.ftd_mps_info(self.h, C.byref(n), bd.ctypes.data_as(_abi.I32P), C.byref(ln),
                               C.byref(pr)))
        return {"n_sites": n.value, "bond_dims": bd[: n.value - 1].tolist(),
                "log_norm": ln.value, "precision": pr.value}

    def site(self, i: int, shape) -> np.ndarray:
        n = int(np.prod(shape))
        buf = np.zeros(2 * n, dtype=np.float64)
        check(lib.ftd_mps_get_site(self.ctx.h, self.h, int(i), _abi._dptr(buf), n))
        return (buf[0::2] + 1j * buf[1::2]).reshape(shape)

    def copy(self):
        h = C.c_void_p()
        check(lib.ftd_mps_copy(self.ctx.h, self.h, C.byref(h)))
        return Mps(self.ctx, h)

    def set_precision(self, precision: str):
        check(lib.ftd_mps_set_precision(self.h, PRECISION[precision]))

    def norm2(self) -> float:
        out = C.c_double()
        check(lib.ftd_mps_norm(self.ctx.h, self.h, C.byref(out)))
        return out.value

    def set_site(self, i: int, tensor):
        """Overwrite site i with a host tensor of the same shape."""
        t = np.ascontiguousarray(np.asarray(tensor, dtype=np.complex128)).reshape(-1)
        buf = np.empty(2 * t.size)
        buf[0::2] = t.real
        buf[1::2] = t.imag
        check(lib.ftd_mps_set_site(self.ctx.h, self.h, int(i), _abi._dptr(buf), t.size))

    def save(self, path: str):
        """Checkpoint the exact tensors, log-norm and precision to a file."""
        check(lib.ftd_mps_save(self.ctx.h, self.h, str(path).encode()))


def mps_load(ctx, path):
    """A state written by Mps.save."""
    out = C.c_void_p()
    check(lib.ftd_mps_load(ctx.h, str(path).encode(), C.byref(out)))
    return Mps(ctx, out)


def _model_struct(model):
    keep = []

    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        if a.size == 0:
            a = np.zeros(1)
        keep.append(a)
        return a.ctypes.data_as(_abi.DP)

    m = _abi.Model(int(model.n_mol), len(model.omega_loc), len(model.omega_nl),
                   int(model.periodic), int(model.levels_loc), int(model.levels_nl),
                   arr(model.omega_loc), arr(model.g_loc), arr(model.omega_nl),
                   arr(model.g_nl), float(model.V), float(model.R), float(model.e0))
    return m, keep


def mpo_build(ctx: Context, model):
    """MPOs of H and of the current j for a workloads.Model."""
    m, keep = _model_struct(model)
    H, J = C.c_void_p(), C.c_void_p()
    check(lib.ftd_mpo_build(ctx.h, C.byref(m), C.byref(H), C.byref(J)))
    return Mpo(ctx, H), Mpo(ctx, J)


def thermal_prep(ctx, H, beta, n_imag, n_grow, D, cutoff=1e-10, precision="c128",
                 tol=1e-14, mmax=40, expand_tol=0.0):
    """(Psi_beta, ln Z); expand_tol > 0 turns on bond expansion up to D in
    the one-site TDVP steps."""
    psi = C.c_void_p()
    logz = C.c_double()
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_thermal_prep(ctx.h, H.h, float(beta), int(n_imag), int(n_grow), int(D),
                               float(cutoff), float(expand_tol), PRECISION[precision],
                               C.byref(ko), C.byref(psi), C.byref(logz)))
    return Mps(ctx, psi), logz.value


def tdvp_step(ctx, H, psi, dt_real=0.0, dt_imag=0.0, tol=1e-14, mmax=40):
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_tdvp_step(ctx.h, H.h, psi.h, float(dt_real), float(dt_imag), C.byref(ko)))


def tdvp_step_expand(ctx, H, psi, D, expand_tol, dt_real=0.0, dt_imag=0.0, tol=1e-14,
                     mmax=40):
    """One TDVP step with bond expansion up to D (threshold expand_tol)."""
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_tdvp_step_expand(ctx.h, H.h, psi.h, float(dt_real), float(dt_imag), int(D),
                                   float(expand_tol), C.byref(ko)))


def tdvp_pair(ctx, H, psi, phi, dt_real=0.0, dt_imag=0.0, tol=1e-14, mmax=40):
    """One TDVP step of psi and of phi, run concurrently on two streams."""
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_tdvp_pair(ctx.h, H.h, psi.h, phi.h, float(dt_real), float(dt_imag),
                            C.byref(ko)))


def apply_compress(ctx, O, psi, D, cutoff=1e-10):
    out = C.c_void_p()
    check(lib.ftd_apply_compress(ctx.h, O.h, psi.h, int(D), float(cutoff), C.byref(out)))
    return Mps(ctx, out)


def pc_stage(ctx, psi, O, phi, c, D, cutoff=1e-10):
    """compress(psi + c O phi, D): one propagation-and-compression stage."""
    cc = np.array([complex(c).real, complex(c).imag])
    out = C.c_void_p()
    check(lib.ftd_pc_stage(ctx.h, psi.h, O.h, phi.h, _abi._dptr(cc), int(D), float(cutoff),
                           C.byref(out)))
    return Mps(ctx, out)


def overlap(ctx, bra, O, ket) -> complex:
    out = np.zeros(2)
    check(lib.ftd_overlap(ctx.h, bra.h, O.h, ket.h, _abi._dptr(out)))
    return complex(out[0], out[1])


def corr_current(ctx, H, J, psi_beta, D, dt, n_steps, cutoff=1e-10, tol=1e-14, mmax=40):
    out = np.zeros(2 * (n_steps + 1))
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_corr_current(ctx.h, H.h, J.h, psi_beta.h, int(D), float(cutoff), float(dt),
                               int(n_steps), C.byref(ko), _abi._dptr(out)))
    return out[0::2] + 1j * out[1::2]


def mobility(C_t, dt, beta, e0=1.0):
    c = np.ascontiguousarray(np.asarray(C_t, dtype=np.complex128))
    buf = np.empty(2 * c.size)
    buf[0::2] = c.real
    buf[1::2] = c.imag
    mu, mu_cm = C.c_double(), C.c_double()
    check(lib.ftd_mobility(_abi._dptr(buf), int(c.size), float(dt), float(beta), float(e0),
                           C.byref(mu), C.byref(mu_cm)))
    return mu.value, mu_cm.value


def mean_free_path(C_t, dt, e0=1.0):
    """(l_mfp, v, tau) from C(t) samples on a uniform grid."""
    c = np.ascontiguousarray(np.asarray(C_t, dtype=np.complex128))
    buf = np.empty(2 * c.size)
    buf[0::2] = c.real
    buf[1::2] = c.imag
    out = [C.c_double() for _ in range(3)]
    check(lib.ftd_mean_free_path(_abi._dptr(buf), int(c.size), float(dt), float(e0),
                                 *[C.byref(o) for o in out]))
    return tuple(o.value for o in out)


def fgr_corr(t, V, omega, g, beta, e0=1.0, R=1.0):
    """Hopping-limit current correlation at times t (complex array)."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    gg = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    out = np.empty(2 * t.size)
    check(lib.ftd_fgr_corr(_abi._dptr(t), int(t.size), _abi._dptr(om), _abi._dptr(gg),
                           int(om.size), float(V), float(beta), float(e0), float(R),
                           _abi._dptr(out)))
    return out[0::2] + 1j * out[1::2]


def mobility_sweep(ctx, model, points, n_imag, n_grow, D, dt, n_steps, cutoff=1e-10,
                   precision="c128", tol=1e-14, mmax=40):
    """Mobility (a.u.) and ln Z for each (beta, V, omega_scale) point; the
    frequency scale s maps omega -> s omega, g -> g / sqrt(s) on every mode."""
    m, keep = _model_struct(model)
    pts = (_abi.SweepPoint * len(points))(*[_abi.SweepPoint(float(b), float(v), float(sc))
                                            for b, v, sc in points])
    mu = np.zeros(len(points))
    logz = np.zeros(len(points))
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_mobility_sweep(ctx.h, C.byref(m), pts, len(points), int(n_imag), int(n_grow),
                                 int(D), float(cutoff), float(dt), int(n_steps),
                                 PRECISION[precision], C.byref(ko), _abi._dptr(mu),
                                 _abi._dptr(logz)))
    return mu, logz


def mobility_grad(ctx, model, beta, n_imag, n_grow, D, dt, n_steps, cutoff=1e-10,
                  precision="c128", tol=1e-14, mmax=40, rel_step=1e-4):
    """(mu, gradients) with gradients a dict of d mu / d omega_loc, g_loc,
    omega_nl, g_nl (arrays), by central finite differences on the GPU."""
    m, keep = _model_struct(model)
    nl, nn = len(model.omega_loc), len(model.omega_nl)
    out = {k: np.zeros(max(1, n)) for k, n in (("omega_loc", nl), ("g_loc", nl),
                                                  ("omega_nl", nn), ("g_nl", nn))}
    mu = C.c_double()
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_mobility_grad(ctx.h, C.byref(m), float(beta), int(n_imag), int(n_grow), int(D),
                                float(cutoff), float(dt), int(n_steps), PRECISION[precision],
                                C.byref(ko), float(rel_step), C.byref(mu),
                                _abi._dptr(out["omega_loc"]), _abi._dptr(out["g_loc"]),
                                _abi._dptr(out["omega_nl"]), _abi._dptr(out["g_nl"])))
    grads = {"omega_loc": out["omega_loc"][:nl], "g_loc": out["g_loc"][:nl],
             "omega_nl": out["omega_nl"][:nn], "g_nl": out["g_nl"][:nn]}
    return mu.value, grads


def mobility_autograd(ctx, model, beta, omega_loc, g_loc, omega_nl, g_nl, n_imag, n_grow, D,
                      dt, n_steps, cutoff=1e-10, precision="c128", tol=1e-14, mmax=40,
                      rel_step=1e-4):
    """The mobility (a.u.) as a differentiable function of the shared mode
    frequencies and couplings, given as torch tensors (float64, CPU; empty
    tensors where the model has no such modes).  The forward pass runs
    ftd_mobility_grad: mu and its gradient, by central finite differences
    through the whole GPU path (relative step rel_step); backward scales that
    gradient by the incoming mu-bar, so the isotope derivative or any chain
    through omega(m), g(m) follows from torch's autograd."""
    return Mobility.apply(omega_loc, g_loc, omega_nl, g_nl, ctx, model, beta,
                          (n_imag, n_grow, D, dt, n_steps, cutoff, precision, tol, mmax,
                           rel_step))


def _mobility_function():
    import torch

    class _Mobility(torch.autograd.Function):
        @staticmethod
        def forward(fctx, omega_loc, g_loc, omega_nl, g_nl, ctx, model, beta, run):
            import dataclasses
            (n_imag, n_grow, D, dt, n_steps, cutoff, precision, tol, mmax, rel_step) = run
            m = dataclasses.replace(
                model, omega_loc=omega_loc.detach().double().tolist(),
                g_loc=g_loc.detach().double().tolist(),
                omega_nl=omega_nl.detach().double().tolist(),
                g_nl=g_nl.detach().double().tolist())
            mu, gr = mobility_grad(ctx, m, beta, n_imag, n_grow, D, dt, n_steps, cutoff=cutoff,
                                   precision=precision, tol=tol, mmax=mmax, rel_step=rel_step)
            grads = [torch.as_tensor(np.asarray(gr[k], dtype=np.float64)).reshape(t.shape)
                     for k, t in (("omega_loc", omega_loc), ("g_loc", g_loc),
                                  ("omega_nl", omega_nl), ("g_nl", g_nl))]
            fctx.save_for_backward(*grads)
            return torch.tensor(mu, dtype=torch.float64)

        @staticmethod
        def backward(fctx, mu_bar):
            gw, gg, gwn, ggn = fctx.saved_tensors
            return (mu_bar * gw, mu_bar * gg, mu_bar * gwn, mu_bar * ggn,
                    None, None, None, None)

    return _Mobility


class _LazyMobility:
    """torch.autograd.Function of the mobility (see mobility_autograd),
    created on first use so that importing the binding does not need torch's
    autograd machinery."""
    _fn = None

    def apply(self, *args):
        if _LazyMobility._fn is None:
            _LazyMobility._fn = _mobility_function()
        return _LazyMobility._fn.apply(*args)


Mobility = _LazyMobility()


def reduced_density(ctx, model, psi):
    """sigma_ij = <psi|c+_j c_i|psi>/<psi|psi> (N x N complex) for a state of `model`."""
    m, keep = _model_struct(model)
    n = int(model.n_mol)
    out = np.empty(2 * n * n)
    check(lib.ftd_reduced_density(ctx.h, C.byref(m), psi.h, _abi._dptr(out)))
    return (out[0::2] + 1j * out[1::2]).reshape(n, n)


def coherent_length(sigma):
    """L = (sum |sigma_ij|)^2 / (N sum |sigma_ij|^2)."""
    s = np.asarray(sigma, dtype=np.complex128)
    n = s.shape[0]
    if s.shape != (n, n):
        raise ValueError("sigma must be square")
    buf = np.empty(2 * n * n)
    buf[0::2] = s.real.reshape(-1)
    buf[1::2] = s.imag.reshape(-1)
    L = C.c_double()
    check(lib.ftd_coherent_length(_abi._dptr(buf), int(n), C.byref(L)))
    return L.value


def qr(ctx, M, lq=False):
    """Device gauge factorisation: (Q, R) with M = Q R, or (L, Q) with M = L Q."""
    M = np.ascontiguousarray(np.asarray(M, dtype=np.complex128))
    rows, cols = M.shape
    k = min(rows, cols)
    buf = np.empty(2 * M.size)
    buf[0::2] = M.real.reshape(-1)
    buf[1::2] = M.imag.reshape(-1)
    q = np.empty(2 * M.size)
    f = np.empty(2 * k * k)
    check(lib.ftd_qr(ctx.h, int(rows), int(cols), _abi._dptr(buf), int(bool(lq)), _abi._dptr(q),
                     _abi._dptr(f)))
    Q = (q[0::2] + 1j * q[1::2]).reshape(rows, cols)
    F = (f[0::2] + 1j * f[1::2]).reshape(k, k)
    return (F, Q) if lq else (Q, F)


def mps_from_host(ctx, tensors, log_norm=0.0, precision="c128"):
    dims = []
    flat = []
    for t in tensors:
        t = np.asarray(t, dtype=np.complex128)
        dims += list(t.shape)
        flat.append(t.reshape(-1))
    x = np.concatenate(flat)
    buf = np.empty(2 * x.size)
    buf[0::2] = x.real
    buf[1::2] = x.imag
    d = np.asarray(dims, dtype=np.int32)
    out = C.c_void_p()
    check(lib.ftd_mps_from_host(ctx.h, len(tensors), d.ctypes.data_as(_abi.I32P),
                                _abi._dptr(buf), float(log_norm), PRECISION[precision],
                                C.byref(out)))
    return Mps(ctx, out)


def gemm(ctx, A, B, transA=0, transB=0, precision="c128"):
    """C = op(A) op(B) on the device (kernel parity tests)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    B = np.ascontiguousarray(np.asarray(B, dtype=np.complex128))
    M = A.shape[0] if transA == 0 else A.shape[1]
    K = A.shape[1] if transA == 0 else A.shape[0]
    N = B.shape[1] if transB == 0 else B.shape[0]
    ab = np.empty(2 * A.size); ab[0::2] = A.real.reshape(-1); ab[1::2] = A.imag.reshape(-1)
    bb = np.empty(2 * B.size); bb[0::2] = B.real.reshape(-1); bb[1::2] = B.imag.reshape(-1)
    cb = np.zeros(2 * M * N)
    check(lib.ftd_gemm(ctx.h, PRECISION[precision], M, N, K, int(transA), int(transB),
                       _abi._dptr(ab), _abi._dptr(bb), _abi._dptr(cb)))
    return (cb[0::2] + 1j * cb[1::2]).reshape(M, N)


def gemm_noalloc(ctx, A, B, C_out, M, N, K, transA=0, transB=0, precision="c128"):
    """ftd_gemm_noalloc on device tensors in split planes (real plane, then
    imaginary plane): A and B float64 (c128) or float32 (c64), C_out float64
    with 2*M*N elements.  Enqueued on the context stream; nothing is
    allocated."""
    import torch
    et = torch.float64 if precision == "c128" else torch.float32
    na = M * K
    nb = K * N
    for name, t, n, dt in (("A", A, 2 * na, et), ("B", B, 2 * nb, et),
                           ("C_out", C_out, 2 * M * N, torch.float64)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name}: need a contiguous {dt} device tensor of {n} elements")
    check(lib.ftd_gemm_noalloc(ctx.h, PRECISION[precision], int(M), int(N), int(K),
                               int(transA), int(transB), C.c_void_p(A.data_ptr()),
                               C.c_void_p(B.data_ptr()), C.c_void_p(C_out.data_ptr())))


def svd_trunc(ctx, T, D, cutoff=1e-10, s_left=True):
    """Truncated SVD on the device: returns (L, R) with T ~ L @ R."""
    T = np.ascontiguousarray(np.asarray(T, dtype=np.complex128))
    M, N = T.shape
    ns = min(M, N)
    tb = np.empty(2 * T.size); tb[0::2] = T.real.reshape(-1); tb[1::2] = T.imag.reshape(-1)
    Lb = np.zeros(2 * M * ns)
    Rb = np.zeros(2 * ns * N)
    k = C.c_int32()
    check(lib.ftd_svd_trunc(ctx.h, M, N, _abi._dptr(tb), int(D), float(cutoff), int(bool(s_left)),
                            _abi._dptr(Lb), _abi._dptr(Rb), C.byref(k)))
    k = k.value
    L = (Lb[0::2] + 1j * Lb[1::2])[: M * k].reshape(M, k)
    R = (Rb[0::2] + 1j * Rb[1::2])[: k * N].reshape(k, N)
    return L, R


def _check_site_vector(H, psi, site, x):
    """The C ABI reads psi's site shape from x without a length: refuse an x
    of another size here (an out-of-range site is left to the library)."""
    dims, _ = H.info()
    L = len(dims)
    if not 0 <= int(site) < L:
        return
    bonds = psi.info()["bond_dims"]
    dl = 1 if site == 0 else bonds[site - 1]
    dr = 1 if site == L - 1 else bonds[site]
    want = dl * int(dims[site]) ** 2 * dr
    if x.size != want:
        raise ValueError(f"site {site} holds {want} elements, x has {x.size}")


def heff_expm(ctx, H, psi, site, x, z, tol=1e-14, mmax=40, n_repeat=1):
    """exp(z H_eff) x at `site` by the library's Krylov exponential; returns
    (y, Krylov vector count)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    _check_site_vector(H, psi, site, x)
    xb = np.empty(2 * x.size)
    xb[0::2] = x.real.reshape(-1)
    xb[1::2] = x.imag.reshape(-1)
    yb = np.zeros_like(xb)
    m = C.c_int32(0)
    ko = _abi._krylov(tol, mmax)
    check(lib.ftd_heff_expm(ctx.h, H.h, psi.h, int(site), _abi._dptr(xb), _abi._dptr(yb),
                            float(complex(z).real), float(complex(z).imag), C.byref(ko),
                            int(n_repeat), C.byref(m)))
    return (yb[0::2] + 1j * yb[1::2]).reshape(x.shape), int(m.value)


def heff_apply(ctx, H, psi, site, x, n_repeat=1):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    _check_site_vector(H, psi, site, x)
    xb = np.empty(2 * x.size)
    xb[0::2] = x.real.reshape(-1)
    xb[1::2] = x.imag.reshape(-1)
    yb = np.zeros_like(xb)
    check(lib.ftd_heff_apply(ctx.h, H.h, psi.h, int(site), _abi._dptr(xb), _abi._dptr(yb),
                             int(n_repeat)))
    return (yb[0::2] + 1j * yb[1::2]).reshape(x.shape)
