"""Explicit operator forms used to pin the oracle on tiny inputs (tests only).

Everything here is built from the paper's definitions, independently of the
oracle's Table 4b double loop:

* sampling operator R(d, t) (Section 3) as a 0/1 matrix in the natural pair
  order (d, t) -> d*|T| + t;
* commutation P and unification Q (Definition 1, Section 4), checked against
  the printed Example by ``test_oracle_pins``;
* the Corollary 1 operators of every pairwise kernel built from P, Q, I, 1 and
  np.kron;
* the Table 4a feature maps for linear base kernels.
"""
from __future__ import annotations

import numpy as np


def sampling_operator(d, t, nd: int, nt: int) -> np.ndarray:
    """R(d, t): row i is the indicator of pair (d_i, t_i) in natural order."""
    R = np.zeros((len(d), nd * nt))
    R[np.arange(len(d)), np.asarray(d) * nt + np.asarray(t)] = 1.0
    return R


def commutation(nd: int, nt: int) -> np.ndarray:
    """P in R^{(T x D) x (D x T)}: P[(t, d), (d, t)] = 1 (Definition 1)."""
    P = np.zeros((nt * nd, nd * nt))
    for d in range(nd):
        for t in range(nt):
            P[t * nd + d, d * nt + t] = 1.0
    return P


def unification(nd: int, nt: int) -> np.ndarray:
    """Q in R^{(D x T) x (D x D)}: Q[(d, t), (d', d'')] = 1 iff d = d' = d'' (Definition 1)."""
    Q = np.zeros((nd * nt, nd * nd))
    for d in range(nd):
        for t in range(nt):
            Q[d * nt + t, d * nd + d] = 1.0
    return Q


def unification_targets(nd: int, nt: int) -> np.ndarray:
    """PQ in R^{(D x T) x (T x T)}: 1 iff t = t' = t'' (values given in Definition 1)."""
    U = np.zeros((nd * nt, nt * nt))
    for d in range(nd):
        for t in range(nt):
            U[d * nt + t, t * nt + t] = 1.0
    return U


def corollary1_operator(kind: str, D: np.ndarray, T: np.ndarray | None = None,
                        antisym_as_printed: bool = False, mlpk_without_transpose: bool = False):
    """The full-domain operator K_kind of Corollary 1 as an explicit matrix.

    Heterogeneous kinds act on D x T pairs (natural order), homogeneous kinds
    on D x D pairs.  ``antisym_as_printed`` uses the printed (P - I) instead of
    the reading (I - P); ``mlpk_without_transpose`` uses the restated form with
    (I - Q) on the right instead of (I - Q)^T.
    """
    m = D.shape[0]
    if kind in ("symmetric", "antisymmetric", "ranking", "mlpk"):
        I = np.eye(m * m)
        P = commutation(m, m)
        DD = np.kron(D, D)
        if kind == "symmetric":
            return (P + I) @ DD
        if kind == "antisymmetric":
            return ((P - I) if antisym_as_printed else (I - P)) @ DD
        if kind == "ranking":
            return (I - P) @ np.kron(D, np.ones((m, m))) @ (I - P)
        Q = unification(m, m)
        right = (I - Q) if mlpk_without_transpose else (I - Q).T
        return (I + P) @ (I - Q) @ DD @ right @ (I + P)
    q = T.shape[0]
    if kind in ("kronecker", "gaussian"):
        return np.kron(D, T)
    if kind == "linear":
        return np.kron(D, np.ones((q, q))) + np.kron(np.ones((m, m)), T)
    if kind == "cartesian":
        return np.kron(D, np.eye(q)) + np.kron(np.eye(m), T)
    if kind == "poly2d":
        Q = unification(m, q)
        PQ = unification_targets(m, q)
        return Q @ np.kron(D, D) @ Q.T + 2.0 * np.kron(D, T) + PQ @ np.kron(T, T) @ PQ.T
    raise ValueError(kind)


def feature_map(kind: str, Xd: np.ndarray, Xt: np.ndarray | None, d, t) -> np.ndarray:
    """Table 4a pair feature vectors for linear base kernels (rows = pairs)."""
    d = np.asarray(d)
    t = np.asarray(t)
    xd = Xd[d]
    if kind in ("symmetric", "antisymmetric", "ranking", "mlpk"):
        xs = Xd[t]
        if kind == "symmetric":
            return np.sqrt(0.5) * (np.einsum("ni,nj->nij", xd, xs) + np.einsum("ni,nj->nij", xs, xd)).reshape(len(d), -1)
        if kind == "antisymmetric":
            return np.sqrt(0.5) * (np.einsum("ni,nj->nij", xd, xs) - np.einsum("ni,nj->nij", xs, xd)).reshape(len(d), -1)
        diff = xd - xs
        if kind == "ranking":
            return diff
        return np.einsum("ni,nj->nij", diff, diff).reshape(len(d), -1)
    xt = Xt[t]
    if kind == "linear":
        return np.concatenate([xd, xt], axis=1)
    if kind == "poly2d":
        z = np.concatenate([xd, xt], axis=1)
        return np.einsum("ni,nj->nij", z, z).reshape(len(d), -1)
    if kind in ("kronecker", "gaussian"):
        return np.einsum("ni,nj->nij", xd, xt).reshape(len(d), -1)
    if kind == "cartesian":
        nd, nt = Xd.shape[0], Xt.shape[0]
        et = np.eye(nt)[t]
        ed = np.eye(nd)[d]
        f1 = np.einsum("ni,nj->nij", xd, et).reshape(len(d), -1)
        f2 = np.einsum("ni,nj->nij", ed, xt).reshape(len(d), -1)
        return np.concatenate([f1, f2], axis=1)
    raise ValueError(kind)
