"""Pins for the oracle's regularized risk (other losses, Section 3) and truncated Newton.

Gradients against central differences of the objective built from the explicit kernel
matrix; the logistic loss against scikit-learn's log loss; the squared-loss solution against
a dense solve of the ridge system; Newton solutions against scipy's optimiser on the explicit
objective."""
import numpy as np
import pytest

import oracle
from oracle import erm

sopt = pytest.importorskip("scipy.optimize")
skm = pytest.importorskip("sklearn.metrics")


def _problem(seed, kind="kronecker", m=8, q=7, n=40):
    r = np.random.default_rng([81, seed])
    Xd, Xt = r.standard_normal((m, 3)), r.standard_normal((q, 3))
    D = np.exp(-((Xd[:, None] - Xd[None]) ** 2).sum(-1) / 4)
    T = np.exp(-((Xt[:, None] - Xt[None]) ** 2).sum(-1) / 4)
    idx = r.choice(m * q, n, replace=False)
    c, e = (idx // q).astype(np.int32), (idx % q).astype(np.int32)
    K = oracle.kernel_matrix(kind, D, T, (c, e), (c, e))
    yb = np.where(r.standard_normal(n) + (Xd[c] * Xt[e]).sum(1) > 0, 1.0, -1.0)
    return D, T, (c, e), K, yb, r


def _explicit_J(K, y, lam, loss):
    def J(a):
        L, _, _ = erm.loss_terms(loss, K @ a, y)
        return L + 0.5 * lam * a @ K @ a
    return J


@pytest.mark.parametrize("loss", ["squared", "logistic", "sqhinge", "hinge"])
def test_gradient_against_central_differences(loss):
    D, T, pairs, K, y, r = _problem(1)
    lam = 0.3
    a = 0.2 * r.standard_normal(len(y))
    J, grad = erm.objective("kronecker", D, T, pairs, y, a, lam, loss)
    Jx = _explicit_J(K, y, lam, loss)
    assert abs(J - Jx(a)) <= 1e-12 * max(1.0, abs(J))
    h = 1e-6
    fd = np.array([(Jx(a + h * ek) - Jx(a - h * ek)) / (2 * h) for ek in np.eye(len(y))])
    # the hinge has kinks: away from them its subgradient is the gradient
    assert np.linalg.norm(grad - fd) <= 1e-6 * np.linalg.norm(fd)


def test_loss_derivatives_and_library_log_loss():
    r = np.random.default_rng(82)
    p = 3 * r.standard_normal(50)
    y = np.where(r.random(50) < 0.5, 1.0, -1.0)
    L, g, d = erm.loss_terms("logistic", p, y)
    prob = 1.0 / (1.0 + np.exp(-p))
    assert abs(L - skm.log_loss((y > 0).astype(int), prob, normalize=False)) < 1e-9
    for loss in ("squared", "logistic", "sqhinge"):
        L, g, d = erm.loss_terms(loss, p, y)
        h = 1e-6
        Lp = np.array([erm.loss_terms(loss, p + h * ek, y)[0] for ek in np.eye(50)])
        Lm = np.array([erm.loss_terms(loss, p - h * ek, y)[0] for ek in np.eye(50)])
        np.testing.assert_allclose(g, (Lp - Lm) / (2 * h), rtol=1e-5, atol=1e-6)
        gp = erm.loss_terms(loss, p + h, y)[1]
        gm = erm.loss_terms(loss, p - h, y)[1]
        # the squared hinge's second derivative jumps at y p = 1
        ok = np.abs(1 - y * p) > 1e-3
        np.testing.assert_allclose(d[ok], ((gp - gm) / (2 * h))[ok], rtol=1e-5, atol=1e-6)


def test_squared_loss_newton_is_the_ridge_solution():
    D, T, pairs, K, _, r = _problem(2)
    y = r.standard_normal(len(pairs[0]))
    lam = 0.5
    res = erm.newton("kronecker", D, T, pairs, y, lam, "squared", max_newton=30, max_cg=200, tol=1e-12)
    ref = np.linalg.solve(K + lam * np.eye(len(y)), y)
    assert np.linalg.norm(res["a"] - ref) / np.linalg.norm(ref) < 1e-8


@pytest.mark.parametrize("loss", ["logistic", "sqhinge"])
@pytest.mark.parametrize("kind", ["kronecker", "symmetric"])
def test_newton_matches_scipy_minimiser(loss, kind):
    if kind == "symmetric":
        r = np.random.default_rng(83)
        X = r.standard_normal((9, 3))
        D = np.exp(-((X[:, None] - X[None]) ** 2).sum(-1) / 4)
        T = None
        c = r.integers(0, 9, 45).astype(np.int32); e = r.integers(0, 9, 45).astype(np.int32)
        pairs = (c, e)
        K = oracle.kernel_matrix(kind, D, T, pairs, pairs)
        y = np.where(r.standard_normal(45) > 0, 1.0, -1.0)
    else:
        D, T, pairs, K, y, _ = _problem(3)
    lam = 0.1
    res = erm.newton(kind, D, T, pairs, y, lam, loss, max_newton=50, max_cg=100, tol=1e-10)
    assert res["gnorm"] <= 1e-10 * res["gnorm0"]
    Jx = _explicit_J(K, y, lam, loss)

    def grad(a):
        _, g, _ = erm.loss_terms(loss, K @ a, y)
        return K @ (g + lam * a)

    opt = sopt.minimize(Jx, np.zeros(len(y)), jac=grad, method="L-BFGS-B",
                        options=dict(gtol=1e-12, ftol=1e-15, maxiter=20000))
    # the same objective value; predictions agree (K may be singular, so compare K a)
    assert abs(Jx(res["a"]) - opt.fun) <= 1e-9 * max(1.0, abs(opt.fun))
    assert Jx(res["a"]) <= opt.fun + 1e-9 * max(1.0, abs(opt.fun))
    np.testing.assert_allclose(K @ res["a"], K @ opt.x, rtol=0, atol=1e-4 * np.abs(K @ opt.x).max())
