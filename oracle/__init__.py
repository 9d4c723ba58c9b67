"""Plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and the GPU library never imports it.

The arithmetic lives in ``gvt_oracle.c`` (plain C, OpenMP over output rows,
``-O2 -ffp-contract=off``).  It evaluates the pairwise kernel functions of
Table 4b by look-ups into the base kernel matrices and sums over all input
pairs with a double loop (Section 4, "approach 1", the standard
matrix-vector product), and solves the ridge system of Section 3 eq. (1) with
textbook conjugate gradients.  This module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gvt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Oracle-private kind codes (must mirror the enum in gvt_oracle.c).
KINDS = {
    "kronecker": 0,
    "gaussian": 0,  # the pairwise Gaussian is the Kronecker kernel of Gaussian bases
    "linear": 1,
    "poly2d": 2,
    "cartesian": 3,
    "symmetric": 4,
    "antisymmetric": 5,
    "ranking": 6,
    "mlpk": 7,
}
HOMOGENEOUS = {"symmetric", "antisymmetric", "ranking", "mlpk"}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = [
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-std=c99", "-Wall", "-o", _LIB, _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_pairwise_matvec.restype = ctypes.c_int
        lib.oracle_pairwise_matvec.argtypes = [
            ctypes.c_int, P, I64, I64, I64, P, I64, I64, I64,
            P, P, I64, P, I64, P, P, I64, P, I64, I64, P, I64, ctypes.c_int,
        ]
        lib.oracle_kernel_matrix.restype = ctypes.c_int
        lib.oracle_kernel_matrix.argtypes = [
            ctypes.c_int, P, I64, I64, I64, P, I64, I64, I64,
            P, P, I64, P, P, I64, P,
        ]
        lib.oracle_krr_cg.restype = ctypes.c_int
        lib.oracle_krr_cg.argtypes = [
            ctypes.c_int, P, I64, I64, I64, P, I64, I64, I64,
            P, P, I64, P, P, I64, I64, ctypes.c_double, P, I64, P, P, P, ctypes.c_int,
        ]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_auc.restype = ctypes.c_double
        lib.oracle_auc.argtypes = [P, P, I64]
        lib.oracle_krr_minres.restype = ctypes.c_int
        lib.oracle_krr_minres.argtypes = [
            ctypes.c_int, P, I64, I64, I64, P, I64, I64, I64,
            P, P, I64, P, P, I64, I64, ctypes.c_double,
            P, P, I64, P, I64, P, I64, P, P, P, P, P, P, P, ctypes.c_int,
        ]
        lib.oracle_base_kernel.restype = ctypes.c_int
        lib.oracle_base_kernel.argtypes = [ctypes.c_int, P, I64, I64, P, I64, I64, I64, ctypes.c_double, P, I64]
        lib.oracle_tanimoto.restype = ctypes.c_int
        lib.oracle_tanimoto.argtypes = [P, I64, I64, P, I64, I64, I64, P, I64]
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


def _bases(kind, D, T):
    D = _f64(D)
    if kind in HOMOGENEOUS or T is None:
        T = D
    else:
        T = _f64(T)
    return D, T


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def pairwise_matvec(kind, D, T, out_pairs, in_pairs, v, rows=None, nthreads=0):
    """u = R(a,b) K_kind R(c,e)^T v by the Table 4b double loop (FP64).

    out_pairs = (a, b), in_pairs = (c, e); v is (n,) or (n, r).  ``rows``
    optionally selects output pairs (row-sampled mode); the result then has
    len(rows) rows in that order.
    """
    lib = _load()
    D, T = _bases(kind, D, T)
    a, b = _i32(out_pairs[0]), _i32(out_pairs[1])
    c, e = _i32(in_pairs[0]), _i32(in_pairs[1])
    v = np.asarray(v, dtype=np.float64)
    squeeze = v.ndim == 1
    V = np.asfortranarray(v.reshape(len(c), -1))
    nrhs = V.shape[1]
    rsel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nev = len(a) if rsel is None else len(rsel)
    U = np.zeros((nev, nrhs), dtype=np.float64, order="F")
    rc = lib.oracle_pairwise_matvec(
        KINDS[kind], _ptr(D), D.shape[0], D.shape[1], D.shape[1],
        _ptr(T), T.shape[0], T.shape[1], T.shape[1],
        _ptr(a), _ptr(b), len(a), _ptr(rsel), 0 if rsel is None else len(rsel),
        _ptr(c), _ptr(e), len(c), _ptr(V), nrhs, max(len(c), 1), _ptr(U), max(nev, 1),
        int(nthreads),
    )
    if rc != 0:
        raise ValueError(f"oracle_pairwise_matvec rejected its arguments (rc={rc})")
    return U[:, 0] if squeeze else U


def kernel_matrix(kind, D, T, out_pairs, in_pairs):
    """Explicit two-sample kernel matrix K[i, j] = k(out_i, in_j) (tiny inputs)."""
    lib = _load()
    D, T = _bases(kind, D, T)
    a, b = _i32(out_pairs[0]), _i32(out_pairs[1])
    c, e = _i32(in_pairs[0]), _i32(in_pairs[1])
    K = np.zeros((len(a), len(c)), dtype=np.float64)
    rc = lib.oracle_kernel_matrix(
        KINDS[kind], _ptr(D), D.shape[0], D.shape[1], D.shape[1],
        _ptr(T), T.shape[0], T.shape[1], T.shape[1],
        _ptr(a), _ptr(b), len(a), _ptr(c), _ptr(e), len(c), _ptr(K),
    )
    if rc != 0:
        raise ValueError("oracle_kernel_matrix rejected its arguments")
    return K


def krr_cg(kind, D, T, pairs, y, lambdas, max_iter=200, tol=1e-6, nthreads=0):
    """Textbook FP64 CG on (K + lambda I) a = y, one solve per lambda.

    Returns (A[n, nlam], iters[nlam], relres_recurrence[nlam], relres_true[nlam]).
    """
    lib = _load()
    D, T = _bases(kind, D, T)
    c, e = _i32(pairs[0]), _i32(pairs[1])
    y = _f64(y)
    lam = _f64(np.atleast_1d(lambdas))
    n, nlam = len(c), len(lam)
    A = np.zeros((n, nlam), dtype=np.float64, order="F")
    iters = np.zeros(nlam, dtype=np.int64)
    rr = np.zeros(nlam)
    rt = np.zeros(nlam)
    rc = lib.oracle_krr_cg(
        KINDS[kind], _ptr(D), D.shape[0], D.shape[1], D.shape[1],
        _ptr(T), T.shape[0], T.shape[1], T.shape[1],
        _ptr(c), _ptr(e), n, _ptr(y), _ptr(lam), nlam, int(max_iter), float(tol),
        _ptr(A), n, _ptr(iters), _ptr(rr), _ptr(rt), int(nthreads),
    )
    if rc == -2:
        raise FloatingPointError("oracle CG breakdown (p.w <= 0 or NaN)")
    if rc != 0:
        raise ValueError("oracle_krr_cg rejected its arguments")
    return A, iters, rr, rt


def base_kernel(kind, X, Y=None, gamma=None):
    """Section 5 base kernel from features (FP64): kind "linear" (<x, y>) or
    "gaussian" (exp(-gamma ||x - y||^2)).  Y=None means Y = X."""
    lib = _load()
    X = _f64(X)
    Y = X if Y is None else _f64(Y)
    assert X.ndim == 2 and Y.ndim == 2 and X.shape[1] == Y.shape[1]
    K = np.zeros((X.shape[0], Y.shape[0]), dtype=np.float64)
    code = {"linear": 0, "gaussian": 1}[kind]
    rc = lib.oracle_base_kernel(code, _ptr(X), X.shape[0], X.shape[1], _ptr(Y), Y.shape[0], Y.shape[1],
                                X.shape[1], float(gamma if gamma is not None else 0.0), _ptr(K),
                                max(Y.shape[0], 1))
    if rc != 0:
        raise ValueError("oracle_base_kernel rejected its arguments")
    return K


def tanimoto(Xbits, Ybits=None, nbits=None):
    """Tanimoto kernel of packed binary vectors (rows of uint64 words, bit b of a row
    in word b // 64 at position b % 64), FP64."""
    lib = _load()
    X = np.ascontiguousarray(Xbits, dtype=np.uint64)
    Y = X if Ybits is None else np.ascontiguousarray(Ybits, dtype=np.uint64)
    nb = 64 * X.shape[1] if nbits is None else int(nbits)
    K = np.zeros((X.shape[0], Y.shape[0]), dtype=np.float64)
    rc = lib.oracle_tanimoto(_ptr(X), X.shape[0], X.shape[1], _ptr(Y), Y.shape[0], Y.shape[1], nb, _ptr(K),
                             max(Y.shape[0], 1))
    if rc != 0:
        raise ValueError("oracle_tanimoto rejected its arguments")
    return K


def auc(p, labels):
    """AUC of predictions against binary labels (> 0.5 positive), ties count 1/2; 0.5
    when one class is empty.  Plain double loop over (positive, negative) pairs."""
    p = _f64(p)
    lab = _f64(labels)
    return float(_load().oracle_auc(_ptr(p), _ptr(lab), len(p)))


def krr_minres(kind, D, T, pairs, y, lambdas, max_iter=200, tol=1e-6, val=None, patience=0,
               nthreads=0):
    """MINRES on (K + lambda I) a = y from a = 0, one solve per lambda, optionally with
    early stopping on a validation sample val = (va, vb, yval_binary).

    Returns a dict: A[n, nlam] (last iterate), A_best[n, nlam] (iterate of the best
    validation AUC), iters, relres_est, relres_true, auc_hist[max_iter, nlam] (NaN past
    the last step), best_iter, best_auc."""
    lib = _load()
    D, T = _bases(kind, D, T)
    c, e = _i32(pairs[0]), _i32(pairs[1])
    y = _f64(y)
    lam = _f64(np.atleast_1d(lambdas))
    n, nlam = len(c), len(lam)
    A = np.zeros((n, nlam), order="F")
    Ab = np.zeros((n, nlam), order="F")
    iters = np.zeros(nlam, dtype=np.int64)
    rr = np.zeros(nlam)
    rt = np.zeros(nlam)
    hist = np.zeros((max(max_iter, 1), nlam))
    bi = np.zeros(nlam, dtype=np.int64)
    ba = np.zeros(nlam)
    if val is not None:
        va, vb, yv = _i32(val[0]), _i32(val[1]), _f64(val[2])
        nval = len(va)
    else:
        va = vb = yv = None
        nval = 0
    rc = lib.oracle_krr_minres(
        KINDS[kind], _ptr(D), D.shape[0], D.shape[1], D.shape[1], _ptr(T), T.shape[0], T.shape[1], T.shape[1],
        _ptr(c), _ptr(e), n, _ptr(y), _ptr(lam), nlam, int(max_iter), float(tol),
        _ptr(va), _ptr(vb), nval, _ptr(yv), int(patience), _ptr(A), n, _ptr(Ab), _ptr(iters), _ptr(rr),
        _ptr(rt), _ptr(hist), _ptr(bi), _ptr(ba), int(nthreads),
    )
    if rc == -2:
        raise FloatingPointError("oracle MINRES breakdown")
    if rc != 0:
        raise ValueError("oracle_krr_minres rejected its arguments")
    return dict(A=A, A_best=Ab, iters=iters, relres_est=rr, relres_true=rt, auc_hist=hist[:max_iter],
                best_iter=bi, best_auc=ba)
