"""Pins for the oracle's MINRES with early stopping and its AUC (no GPU).

MINRES iterates are fixed by their definition: a_k minimises ||y - A a|| over the
Krylov space K_k(A, y), checked by brute force (an orthonormal Krylov basis and a least
squares solve) and against scipy's minres on the explicit matrix; the AUC against
scikit-learn and a hand count; early stopping against its definition replayed step by
step."""
import numpy as np
import pytest

import oracle

spla = pytest.importorskip("scipy.sparse.linalg")
skm = pytest.importorskip("sklearn.metrics")


def _problem(seed, m=9, q=7, n=45, kind="kronecker"):
    r = np.random.default_rng([61, seed])
    Xd, Xt = r.standard_normal((m, 3)), r.standard_normal((q, 3))
    D = np.exp(-((Xd[:, None] - Xd[None]) ** 2).sum(-1) / 4)
    T = np.exp(-((Xt[:, None] - Xt[None]) ** 2).sum(-1) / 4)
    idx = r.choice(m * q, n, replace=False)
    c, e = (idx // q).astype(np.int32), (idx % q).astype(np.int32)
    y = r.standard_normal(n)
    K = oracle.kernel_matrix(kind, D, T, (c, e), (c, e))
    return D, T, c, e, y, K, r


def test_auc_hand_counted_and_sklearn():
    p = np.array([0.9, 0.1, 0.4, 0.4, 0.7])
    lab = np.array([1, 0, 1, 0, 0])
    # positives 0.9, 0.4 against negatives 0.1, 0.4, 0.7: 0.9 beats 3; 0.4 beats 0.1, ties 0.4
    assert oracle.auc(p, lab) == (3 + 1 + 0.5) / 6
    r = np.random.default_rng(62)
    for _ in range(5):
        p = np.round(r.standard_normal(200), 1)  # many ties
        lab = (r.random(200) < 0.3).astype(float)
        assert abs(oracle.auc(p, lab) - skm.roc_auc_score(lab, p)) < 1e-14
    assert oracle.auc(p, np.zeros(200)) == 0.5


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_minres_iterate_is_the_krylov_minimiser(k):
    D, T, c, e, y, K, _ = _problem(k)
    lam = 0.3
    A = K + lam * np.eye(len(y))
    res = oracle.krr_minres("kronecker", D, T, (c, e), y, [lam], max_iter=k, tol=0.0)
    a = res["A"][:, 0]
    assert res["iters"][0] == k
    # orthonormal Krylov basis by modified Gram-Schmidt, then least squares over it
    Q = np.zeros((len(y), k))
    v = y / np.linalg.norm(y)
    for j in range(k):
        Q[:, j] = v
        w = A @ v
        for i in range(j + 1):
            w -= (Q[:, i] @ w) * Q[:, i]
        v = w / np.linalg.norm(w)
    z, *_ = np.linalg.lstsq(A @ Q, y, rcond=None)
    np.testing.assert_allclose(a, Q @ z, rtol=1e-8, atol=1e-10)
    # |phibar_k| is the residual norm of the iterate
    assert abs(res["relres_est"][0] - np.linalg.norm(y - A @ a) / np.linalg.norm(y)) < 1e-10
    assert abs(res["relres_true"][0] - np.linalg.norm(y - A @ a) / np.linalg.norm(y)) < 1e-12


@pytest.mark.parametrize("kind", ["kronecker", "poly2d"])
def test_minres_matches_scipy_and_dense_solve(kind):
    D, T, c, e, y, K, _ = _problem(3, kind=kind)
    lams = [1e-2, 1.0]
    for k in (3, 12):
        res = oracle.krr_minres(kind, D, T, (c, e), y, lams, max_iter=k, tol=0.0)
        for l, lam in enumerate(lams):
            x, _ = spla.minres(K + lam * np.eye(len(y)), y, maxiter=k, rtol=0.0)
            np.testing.assert_allclose(res["A"][:, l], x, rtol=1e-9, atol=1e-9 * np.abs(x).max())
    res = oracle.krr_minres(kind, D, T, (c, e), y, lams, max_iter=500, tol=1e-12)
    for l, lam in enumerate(lams):
        ref = np.linalg.solve(K + lam * np.eye(len(y)), y)
        assert res["relres_true"][l] < 1e-11
        assert np.linalg.norm(res["A"][:, l] - ref) / np.linalg.norm(ref) < 1e-8


def test_early_stopping_follows_its_definition():
    D, T, c, e, y, K, r = _problem(5, m=12, q=10, n=80)
    # validation pairs: other cells of the grid, binary labels from a smooth signal
    rest = np.setdiff1d(np.arange(12 * 10), c.astype(np.int64) * 10 + e)
    vi = r.choice(rest, 30, replace=False)
    va, vb = (vi // 10).astype(np.int32), (vi % 10).astype(np.int32)
    yv = (r.standard_normal(30) > 0).astype(float)
    lams = [1e-3, 0.5]
    pat = 3
    res = oracle.krr_minres("kronecker", D, T, (c, e), y, lams, max_iter=25, tol=0.0, val=(va, vb, yv),
                            patience=pat)
    for l, lam in enumerate(lams):
        best, kbest, ab = 0.5, 0, np.zeros(len(y))
        it = int(res["iters"][l])
        for k in range(1, it + 1):
            ak = oracle.krr_minres("kronecker", D, T, (c, e), y, [lam], max_iter=k, tol=0.0)["A"][:, 0]
            pv = oracle.pairwise_matvec("kronecker", D, T, (va, vb), (c, e), ak)
            auc = skm.roc_auc_score(yv, pv)
            assert abs(res["auc_hist"][k - 1, l] - auc) < 1e-12
            if auc > best + 1e-15:
                best, kbest, ab = auc, k, ak
        assert np.all(np.isnan(res["auc_hist"][it:, l]))
        assert res["best_iter"][l] == kbest and abs(res["best_auc"][l] - best) < 1e-12
        np.testing.assert_allclose(res["A_best"][:, l], ab, rtol=1e-12, atol=1e-14)
        assert it == 25 or it - kbest == pat
