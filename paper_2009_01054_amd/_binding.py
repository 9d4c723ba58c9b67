"""ctypes marshalling for libgvt.so (no computation here)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libgvt.so")

F64, F32, BF16X3, BF16X6 = 0, 1, 2, 3
FLAG_SYMMETRIC_BASES, FLAG_ORDER_A, FLAG_ORDER_B = 1, 2, 4
FLAG_DENSE_TILES, FLAG_NO_DENSE_TILES = 8, 16
KINDS = {
    "kronecker": 0,
    "gaussian": 0,
    "linear": 1,
    "poly2d": 2,
    "cartesian": 3,
    "symmetric": 4,
    "antisymmetric": 5,
    "ranking": 6,
    "mlpk": 7,
}
NOT_CONVERGED = 1

_lib = None


class GvtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgvt error {code}: {msg}")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_2009_01054_amd.build` "
            "(there is no CPU fallback)"
        )
    lib = ctypes.CDLL(_LIB_PATH)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.gvt_last_error.restype = ctypes.c_char_p
    lib.gvt_version.restype = I
    lib.gvt_plan_create.argtypes = [ctypes.POINTER(P), P, I, I64, I64, I64, I64, P, P, I64, P, P, I64, I, P]
    lib.gvt_plan_destroy.argtypes = [P]
    lib.gvt_plan_execute.argtypes = [P, I, P, I64, P, I64, P, I64, I64, P, I64, P]
    lib.gvt_matvec.argtypes = [I, P, I64, I64, I64, P, I64, I64, I64, P, P, I64, P, P, I64, P, I64, I64, P, I64, P]
    lib.gvt_pairwise_matvec.argtypes = [I, P, I, P, I64, I64, I64, P, I64, I64, I64, P, P, I64, P, P, I64,
                                        P, I64, I64, P, I64, I, P]
    lib.gvt_dense_matvec.argtypes = [I, P, I64, I64, I64, P, I64, I64, I64, P, I64, P, I64, P]
    lib.gvt_dense_matvec_noalloc.argtypes = [I, P, I64, I64, I64, P, I64, I64, I64, P, I64, P, I64, P]
    lib.gvt_base_kernel.argtypes = [I, I, P, I64, I64, P, I64, I64, I64, ctypes.c_double, P, I64, P]
    lib.gvt_erm_objective.argtypes = [I, I, P, I64, I64, P, I64, I64, P, P, I64, P, P, ctypes.c_double, P, P, P]
    lib.gvt_erm_newton.argtypes = [I, I, P, I64, I64, P, I64, I64, P, P, I64, P, ctypes.c_double, P, I, I,
                                   ctypes.c_double, I, P, P, P, P, P, P]
    lib.gvt_krr_minres.argtypes = [I, P, I64, I64, P, I64, I64, P, P, I64, P, P, I, P, I64, I, ctypes.c_double,
                                   I, P, I, P, P, P, P, P, P]
    lib.gvt_tanimoto_kernel.argtypes = [I, P, I64, I64, P, I64, I64, I64, P, I64, P]
    lib.gvt_dense_matvec_checked.argtypes = [I, P, I64, I64, I64, P, I64, I64, I64, P, I64, P, I64,
                                             ctypes.c_double, P, P, P]
    lib.gvt_krr_cg.argtypes = [I, P, I64, I64, P, I64, I64, P, P, I64, P, P, I, P, I64, P, I64, I,
                               ctypes.c_double, I, I, P, P, P]
    lib.gvt_krr_cg_batched.argtypes = [I, P, I, P, I, I, ctypes.c_double, I, I, P, P, P]
    lib.gvt_plan_profile.argtypes = [P, I, P, I64, P, I64, P, I64, I64, P, I64, I, P, P]
    lib.gvt_plan_info.argtypes = [P, P]
    lib.gvt_plan_uses_tiles.argtypes = [P, I]
    lib.gvt_empty_cache.argtypes = [P]
    for f in ("gvt_plan_profile", "gvt_plan_info", "gvt_plan_uses_tiles", "gvt_plan_create", "gvt_plan_destroy", "gvt_plan_execute", "gvt_matvec",
              "gvt_pairwise_matvec", "gvt_dense_matvec", "gvt_dense_matvec_noalloc", "gvt_dense_matvec_checked", "gvt_base_kernel", "gvt_tanimoto_kernel", "gvt_krr_minres", "gvt_erm_objective", "gvt_erm_newton", "gvt_krr_cg", "gvt_krr_cg_batched", "gvt_empty_cache"):
        getattr(lib, f).restype = I
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise GvtError(rc, load_library().gvt_last_error().decode())
    return rc


def gvt_last_error() -> str:
    return load_library().gvt_last_error().decode()


def gvt_version() -> int:
    return int(load_library().gvt_version())


def gvt_empty_cache() -> int:
    """Free the library's cached device blocks and staging buffer; returns the
    device bytes freed."""
    lib = load_library()
    freed = ctypes.c_int64(0)
    _check(lib.gvt_empty_cache(ctypes.byref(freed)))
    return int(freed.value)


# ------------------------------------------------------------------ helpers
def _torch():
    import torch

    return torch


def _stream_handle(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _ld(t):
    """Row stride of a row-major 2-D tensor (elements)."""
    assert t.dim() == 2, "expected a 2-D tensor"
    if t.numel() == 0:
        return max(t.shape[1], 1)
    assert t.stride(1) == 1 or t.shape[1] == 1, "base matrices must be row-major (stride(1) == 1)"
    return max(t.stride(0), t.shape[1], 1)


def _idx(x):
    torch = _torch()
    assert x.dtype == torch.int32 and x.is_cuda and x.is_contiguous(), "indices: contiguous int32 device tensors"
    return x


def _prec_of(dtype, prec):
    torch = _torch()
    if prec is not None:
        return prec
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype}")


def _colmajor(V):
    """(n,) or (n, r) tensor -> column-major (n, r) view/copy and ld."""
    V2 = V.reshape(-1, 1) if V.dim() == 1 else V
    if V2.stride(0) != 1:
        V2 = V2.t().contiguous().t()
    return V2, max(V2.stride(1) if V2.shape[1] > 1 else V2.shape[0], 1)


def _kind_codes(kinds):
    if isinstance(kinds, (str, int)):
        kinds = [kinds]
    return [KINDS[k] if isinstance(k, str) else int(k) for k in kinds]


# --------------------------------------------------------------------- plans
class Plan:
    """Owning wrapper of a gvt_plan_t."""

    def __init__(self, handle, nkinds, n_out, n_in):
        self.handle = handle
        self.nkinds = nkinds
        self.n_out = n_out
        self.n_in = n_in

    def execute(self, D, T, V, prec=None, out=None):
        return gvt_plan_execute(self, D, T, V, prec=prec, out=out)

    def close(self):
        if self.handle:
            gvt_plan_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gvt_plan_create(kinds, d_shape, t_shape, out_pairs, in_pairs, flags=0):
    lib = load_library()
    codes = _kind_codes(kinds)
    karr = (ctypes.c_int * len(codes))(*codes)
    a, b = _idx(out_pairs[0]), _idx(out_pairs[1])
    c, e = _idx(in_pairs[0]), _idx(in_pairs[1])
    h = ctypes.c_void_p(0)
    _check(lib.gvt_plan_create(ctypes.byref(h), karr, len(codes), d_shape[0], d_shape[1], t_shape[0],
                               t_shape[1], _ptr(a), _ptr(b), a.numel(), _ptr(c), _ptr(e), c.numel(),
                               int(flags), _stream_handle()))
    return Plan(h, len(codes), a.numel(), c.numel())


def gvt_plan_destroy(plan: Plan):
    lib = load_library()
    h, plan.handle = plan.handle, None
    _check(lib.gvt_plan_destroy(h))


def gvt_plan_execute(plan: Plan, D, T, V, prec=None, out=None):
    """Returns U of shape (nkinds, n_out, nrhs) (squeezed like V)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(D.dtype, prec)
    V2, ldv = _colmajor(V)
    nrhs = V2.shape[1]
    U = out if out is not None else torch.empty((plan.nkinds, nrhs, max(plan.n_out, 1)),
                                                 dtype=D.dtype, device=D.device)
    ldu = U.shape[2]
    _check(lib.gvt_plan_execute(plan.handle, p, _ptr(D), _ld(D), _ptr(T), _ld(T) if T is not None else 0,
                                _ptr(V2), nrhs, ldv, _ptr(U), ldu, _stream_handle()))
    res = U[:, :, : plan.n_out].transpose(1, 2)
    if V.dim() == 1:
        res = res[:, :, 0]
    return res


def gvt_plan_profile(plan: Plan, D, T, V, prec=None, reps=10, out=None):
    """Mean ms per stage group: [prep, stage1, stage2, other] (see gvt.h)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(D.dtype, prec)
    V2, ldv = _colmajor(V)
    nrhs = V2.shape[1]
    U = out if out is not None else torch.empty((plan.nkinds, nrhs, max(plan.n_out, 1)),
                                                 dtype=D.dtype, device=D.device)
    ms = np.zeros(4, dtype=np.float64)
    _check(lib.gvt_plan_profile(plan.handle, p, _ptr(D), _ld(D), _ptr(T), _ld(T) if T is not None else 0,
                                _ptr(V2), nrhs, ldv, _ptr(U), U.shape[2], int(reps),
                                ms.ctypes.data_as(ctypes.c_void_p), _stream_handle()))
    return ms


def gvt_plan_uses_tiles(plan: Plan, prec) -> bool:
    """Whether products of the plan in precision prec run as dense tiles."""
    return bool(_check(load_library().gvt_plan_uses_tiles(plan.handle, int(prec))))


def gvt_plan_info(plan: Plan):
    lib = load_library()
    info = np.zeros(11, dtype=np.float64)
    _check(lib.gvt_plan_info(plan.handle, info.ctypes.data_as(ctypes.c_void_p)))
    keys = ["cost_fma", "dense", "terms", "sbufs", "s_rows", "s_keys", "s_key", "uniq_a", "uniq_b",
            "uniq_c", "uniq_e"]
    return dict(zip(keys, info.tolist()))


# ------------------------------------------------------------- one-shot calls
def gvt_matvec(M, N, out_pairs, in_pairs, V, prec=None):
    torch = _torch()
    lib = load_library()
    p = _prec_of(M.dtype, prec)
    a, b = _idx(out_pairs[0]), _idx(out_pairs[1])
    c, e = _idx(in_pairs[0]), _idx(in_pairs[1])
    V2, ldv = _colmajor(V)
    nrhs = V2.shape[1]
    U = torch.empty((nrhs, max(a.numel(), 1)), dtype=M.dtype, device=M.device)
    _check(lib.gvt_matvec(p, _ptr(M), M.shape[0], M.shape[1], _ld(M), _ptr(N), N.shape[0], N.shape[1],
                          _ld(N), _ptr(a), _ptr(b), a.numel(), _ptr(c), _ptr(e), c.numel(), _ptr(V2),
                          nrhs, ldv, _ptr(U), U.shape[1], _stream_handle()))
    U = U[:, : a.numel()].t()
    return U[:, 0] if V.dim() == 1 else U


def gvt_pairwise_matvec(kinds, D, T, out_pairs, in_pairs, V, prec=None, flags=0):
    """Returns U of shape (nkinds, n_out[, nrhs])."""
    torch = _torch()
    lib = load_library()
    codes = _kind_codes(kinds)
    karr = (ctypes.c_int * len(codes))(*codes)
    p = _prec_of(D.dtype, prec)
    a, b = _idx(out_pairs[0]), _idx(out_pairs[1])
    c, e = _idx(in_pairs[0]), _idx(in_pairs[1])
    V2, ldv = _colmajor(V)
    nrhs = V2.shape[1]
    Tm = T if T is not None else D
    U = torch.empty((len(codes), nrhs, max(a.numel(), 1)), dtype=D.dtype, device=D.device)
    _check(lib.gvt_pairwise_matvec(p, karr, len(codes), _ptr(D), D.shape[0], D.shape[1], _ld(D),
                                   _ptr(Tm), Tm.shape[0], Tm.shape[1], _ld(Tm), _ptr(a), _ptr(b),
                                   a.numel(), _ptr(c), _ptr(e), c.numel(), _ptr(V2), nrhs, ldv,
                                   _ptr(U), U.shape[2], int(flags), _stream_handle()))
    res = U[:, :, : a.numel()].transpose(1, 2)
    return res[:, :, 0] if V.dim() == 1 else res


def gvt_dense_matvec(M, N, Vmat, prec=None, out=None):
    """Umat = M Vmat N^T on matrix cores (complete data)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(M.dtype, prec)
    U = out if out is not None else torch.empty((M.shape[0], N.shape[0]), dtype=M.dtype, device=M.device)
    _check(lib.gvt_dense_matvec(p, _ptr(M), M.shape[0], M.shape[1], _ld(M), _ptr(N), N.shape[0],
                                N.shape[1], _ld(N), _ptr(Vmat), _ld(Vmat), _ptr(U), _ld(U),
                                _stream_handle()))
    return U


BASE_KINDS = {"linear": 0, "gaussian": 1}


def gvt_base_kernel(kind, X, Y=None, gamma=0.0, out=None):
    """Base kernel matrix K[i, j] = k(X_i, Y_j) from features (Section 5): "linear" or
    "gaussian" (exp(-gamma ||x - y||^2)); Y=None gives the exactly symmetric K of X.
    Precision follows X's dtype (float64 / float32)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(X.dtype, None)
    ny = X.shape[0] if Y is None else Y.shape[0]
    K = out if out is not None else torch.empty((X.shape[0], ny), dtype=X.dtype, device=X.device)
    _check(lib.gvt_base_kernel(BASE_KINDS[kind], p, _ptr(X), X.shape[0], _ld(X), _ptr(Y),
                               ny, _ld(Y) if Y is not None else 0, X.shape[1], float(gamma), _ptr(K), _ld(K),
                               _stream_handle()))
    return K


def gvt_tanimoto_kernel(Xbits, Ybits=None, nbits=None, dtype=None, out=None):
    """Tanimoto kernel of packed binary vectors (int64 device tensors of 64-bit words,
    bit b of a row in word b // 64 at position b % 64).  Ybits=None: Y = X."""
    torch = _torch()
    lib = load_library()
    dtype = dtype or torch.float64
    nb = 64 * Xbits.shape[1] if nbits is None else int(nbits)
    ny = Xbits.shape[0] if Ybits is None else Ybits.shape[0]
    K = out if out is not None else torch.empty((Xbits.shape[0], ny), dtype=dtype, device=Xbits.device)
    _check(lib.gvt_tanimoto_kernel(_prec_of(dtype, None), _ptr(Xbits), Xbits.shape[0], _ld(Xbits), _ptr(Ybits),
                                   ny, _ld(Ybits) if Ybits is not None else 0, nb, _ptr(K), _ld(K),
                                   _stream_handle()))
    return K


def gvt_dense_matvec_checked(M, N, Vmat, prec=None, max_relerr=1e-5, out=None):
    """Umat = M Vmat N^T with its error estimated on sampled rows against FP64 and the
    precision raised (bf16x3 -> bf16x6 -> f32) until the estimate is within half of
    max_relerr.  Returns (Umat, estimated relative error, precision used, status)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(M.dtype, prec)
    U = out if out is not None else torch.empty((M.shape[0], N.shape[0]), dtype=M.dtype, device=M.device)
    est = ctypes.c_double(0.0)
    used = ctypes.c_int(0)
    rc = _check(lib.gvt_dense_matvec_checked(p, _ptr(M), M.shape[0], M.shape[1], _ld(M), _ptr(N), N.shape[0],
                                             N.shape[1], _ld(N), _ptr(Vmat), _ld(Vmat), _ptr(U), _ld(U),
                                             float(max_relerr), ctypes.byref(est), ctypes.byref(used),
                                             _stream_handle()))
    return U, est.value, used.value, rc


def gvt_dense_matvec_noalloc(M, N, Vmat, prec=None, out=None):
    """Umat = M Vmat N^T like gvt_dense_matvec, with the library's static per-device
    workspace instead of an allocation (calls on one device must not overlap)."""
    torch = _torch()
    lib = load_library()
    p = _prec_of(M.dtype, prec)
    U = out if out is not None else torch.empty((M.shape[0], N.shape[0]), dtype=M.dtype, device=M.device)
    _check(lib.gvt_dense_matvec_noalloc(p, _ptr(M), M.shape[0], M.shape[1], _ld(M), _ptr(N), N.shape[0],
                                        N.shape[1], _ld(N), _ptr(Vmat), _ld(Vmat), _ptr(U), _ld(U),
                                        _stream_handle()))
    return U


LOSSES = {"squared": 0, "logistic": 1, "sqhinge": 2, "hinge": 3}


def gvt_erm_objective(kind, loss, D, T, pairs, y, a, lam, grad=True):
    """Regularized risk J(a) = L(K a, y) + (lam/2) a^T K a and its (sub)gradient K (g + lam a).
    Returns (J, grad tensor or None)."""
    torch = _torch()
    lib = load_library()
    c, e = _idx(pairs[0]), _idx(pairs[1])
    Tm = T if T is not None else D
    g = torch.empty_like(a) if grad else None
    J = ctypes.c_double(0.0)
    _check(lib.gvt_erm_objective(_kind_codes(kind)[0], LOSSES[loss], _ptr(D), D.shape[0], _ld(D), _ptr(Tm),
                                 Tm.shape[0], _ld(Tm), _ptr(c), _ptr(e), c.numel(), _ptr(y), _ptr(a), float(lam),
                                 _ptr(g), ctypes.byref(J), _stream_handle()))
    return J.value, g


def gvt_erm_newton(kind, loss, D, T, pairs, y, lam, max_newton=20, max_cg=50, tol=1e-8, matvec_prec=F64):
    """Truncated Newton for the regularized risk from a = 0.  Returns a dict with a, steps,
    cg_iters, J, gnorm, gnorm0 and status."""
    torch = _torch()
    lib = load_library()
    c, e = _idx(pairs[0]), _idx(pairs[1])
    Tm = T if T is not None else D
    a = torch.empty(c.numel(), dtype=torch.float64, device=D.device)
    st, cg = ctypes.c_int(0), ctypes.c_int(0)
    J, gn, g0 = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    rc = _check(lib.gvt_erm_newton(_kind_codes(kind)[0], LOSSES[loss], _ptr(D), D.shape[0], _ld(D), _ptr(Tm),
                                   Tm.shape[0], _ld(Tm), _ptr(c), _ptr(e), c.numel(), _ptr(y), float(lam), _ptr(a),
                                   int(max_newton), int(max_cg), float(tol), int(matvec_prec), ctypes.byref(st),
                                   ctypes.byref(cg), ctypes.byref(J), ctypes.byref(gn), ctypes.byref(g0),
                                   _stream_handle()))
    return dict(a=a, steps=st.value, cg_iters=cg.value, J=J.value, gnorm=gn.value, gnorm0=g0.value, status=rc)


class _Validation(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("labels", ctypes.c_void_p), ("patience", ctypes.c_int64)]


def gvt_krr_minres(kind, D, T, pairs, y, lambdas, max_iter=200, tol=1e-6, matvec_prec=F64, val=None,
                   patience=0, check_every=8, history=False):
    """Ridge regression by MINRES from a = 0 (all lambdas share one Lanczos basis), optionally
    with early stopping on a validation sample val = (a, b, labels) (device tensors; labels
    double, > 0.5 positive).  Returns a dict with A[n, nlam] (the best-AUC iterate with
    validation, else the last), iters, relres (true), best_iter, best_auc, auc_hist
    ([max_iter, nlam] when history=True) and status."""
    torch = _torch()
    lib = load_library()
    code = _kind_codes(kind)[0]
    c, e = _idx(pairs[0]), _idx(pairs[1])
    lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
    nlam = len(lam)
    n = c.numel()
    A = torch.empty((nlam, n), dtype=torch.float64, device=D.device)
    iters = np.zeros(nlam, dtype=np.int64)
    rel = np.zeros(nlam)
    bi = np.zeros(nlam, dtype=np.int64)
    ba = np.zeros(nlam)
    hist = np.zeros((max_iter, nlam)) if history else None
    Tm = T if T is not None else D
    vs = None
    if val is not None:
        va, vb, lab = _idx(val[0]), _idx(val[1]), val[2]
        assert lab.dtype == torch.float64 and lab.is_cuda and lab.numel() == va.numel()
        vs = _Validation(va.data_ptr(), vb.data_ptr(), va.numel(), lab.data_ptr(), int(patience))
    rc = lib.gvt_krr_minres(code, _ptr(D), D.shape[0], _ld(D), _ptr(Tm), Tm.shape[0], _ld(Tm), _ptr(c), _ptr(e),
                            n, _ptr(y), lam.ctypes.data_as(ctypes.c_void_p), nlam, _ptr(A), A.stride(0),
                            int(max_iter), float(tol), int(matvec_prec),
                            ctypes.byref(vs) if vs is not None else None, int(check_every),
                            iters.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p),
                            bi.ctypes.data_as(ctypes.c_void_p), ba.ctypes.data_as(ctypes.c_void_p),
                            hist.ctypes.data_as(ctypes.c_void_p) if hist is not None else None,
                            _stream_handle())
    _check(rc)
    return dict(A=A.t(), iters=iters, relres=rel, best_iter=bi, best_auc=ba, auc_hist=hist, status=rc)


class _KrrProblem(ctypes.Structure):
    _fields_ = [("D", ctypes.c_void_p), ("d", ctypes.c_int64), ("ldd", ctypes.c_int64),
                ("T", ctypes.c_void_p), ("t", ctypes.c_int64), ("ldt", ctypes.c_int64),
                ("c", ctypes.c_void_p), ("e", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("y", ctypes.c_void_p), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("A0", ctypes.c_void_p), ("lda0", ctypes.c_int64)]


def gvt_krr_cg_batched(kind, problems, lambdas, max_iter=200, tol=1e-6, matvec_prec=F64,
                       check_every=8):
    """Many ridge problems at once.  problems: sequence of dicts with D, T (None for
    homogeneous kinds), c, e, y and optionally A0 ([n, nlam] view with unit row stride).
    Returns (list of A[n, nlam], iters[nprob, nlam], true_relres[nprob, nlam], status)."""
    torch = _torch()
    lib = load_library()
    code = _kind_codes(kind)[0]
    lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
    nlam = len(lam)
    arr = (_KrrProblem * len(problems))()
    outs, keep = [], []
    for k, pr in enumerate(problems):
        D = pr["D"]
        Tm = pr.get("T") if pr.get("T") is not None else D
        c, e = _idx(pr["c"]), _idx(pr["e"])
        n = c.numel()
        A = torch.empty((nlam, n), dtype=torch.float64, device=D.device)
        outs.append(A)
        A0 = pr.get("A0")
        if A0 is not None and A0.stride(0) != 1:
            A0 = A0.t().contiguous().t()  # column-major n x nlam
        keep.append(A0)  # alive until the call returns
        arr[k] = _KrrProblem(D.data_ptr(), D.shape[0], _ld(D), Tm.data_ptr(), Tm.shape[0], _ld(Tm),
                             c.data_ptr(), e.data_ptr(), n, pr["y"].data_ptr(), A.data_ptr(), n,
                             A0.data_ptr() if A0 is not None else None,
                             A0.stride(1) if A0 is not None else n)
    iters = np.zeros((len(problems), nlam), dtype=np.int64)
    rel = np.zeros((len(problems), nlam), dtype=np.float64)
    rc = lib.gvt_krr_cg_batched(code, ctypes.cast(arr, ctypes.c_void_p), len(problems),
                                lam.ctypes.data_as(ctypes.c_void_p), nlam, int(max_iter), float(tol),
                                int(matvec_prec), int(check_every), iters.ctypes.data_as(ctypes.c_void_p),
                                rel.ctypes.data_as(ctypes.c_void_p), _stream_handle())
    _check(rc)
    return [A.t() for A in outs], iters, rel, rc


def gvt_krr_cg(kind, D, T, pairs, y, lambdas, max_iter=200, tol=1e-6, matvec_prec=F64,
               check_every=8, A0=None, out=None):
    """Ridge CG.  Returns (A[n, nlam], iters[nlam], true_relres[nlam], status)."""
    torch = _torch()
    lib = load_library()
    code = _kind_codes(kind)[0]
    c, e = _idx(pairs[0]), _idx(pairs[1])
    lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
    nlam = len(lam)
    n = c.numel()
    A = out if out is not None else torch.empty((nlam, n), dtype=torch.float64, device=D.device)
    iters = np.zeros(nlam, dtype=np.int64)
    rel = np.zeros(nlam, dtype=np.float64)
    Tm = T if T is not None else D
    A0p = _ptr(A0) if A0 is not None else ctypes.c_void_p(0)
    lda0 = A0.stride(0) if A0 is not None else n
    rc = lib.gvt_krr_cg(code, _ptr(D), D.shape[0], _ld(D), _ptr(Tm), Tm.shape[0], _ld(Tm), _ptr(c), _ptr(e),
                        n, _ptr(y), lam.ctypes.data_as(ctypes.c_void_p), nlam, _ptr(A), A.stride(0), A0p,
                        lda0, int(max_iter), float(tol), int(matvec_prec), int(check_every),
                        iters.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p),
                        _stream_handle())
    _check(rc)
    return A.t(), iters, rel, rc
