"""Regularized kernel risk minimisation beyond ridge regression (test infrastructure only).

Section 3 states the learning problem as min_f L(p, y) + (lambda/2) ||f||^2 over the
RKHS of the pairwise kernel, with predictions p = K a by the representer theorem, and notes
that the GVT speeds up any optimiser dominated by products with K, naming the truncated
Newton method; the conclusions (Section 7) name kernel logistic regression and support
vector machines.  In dual coefficients the objective is

    J(a) = L(K a, y) + (lambda / 2) a^T K a,      grad J = K (g + lambda a),

with g = dL/dp.  Losses (y in {-1, +1} for the classification losses):

    squared        L = 1/2 sum (y - p)^2             g = p - y
    logistic       L = sum log(1 + exp(-y p))        g = -y sigma(-y p)
    squared hinge  L = 1/2 sum max(0, 1 - y p)^2     g = -y max(0, 1 - y p)
    hinge          L = sum max(0, 1 - y p)           subgradient g = -y [y p < 1]

(the squared loss carries 1/2, so its stationary point is the ridge system of eq. (1),
(K + lambda I) a = y, with the same lambda).  The (generalised) Hessian is
K D K + lambda K with D = diag(d), d = d^2L/dp^2: 1, sigma(yp) sigma(-yp), [y p < 1].

Truncated Newton: the Newton equation K (D K + lambda I) delta = -grad J is met by any
delta with (D K + lambda I) delta = -(g + lambda a).  That operator is self-adjoint and
positive in the K inner product <x, y>_K = x^T K y, so each step runs conjugate gradients on
it in that inner product: <z, A z>_K = (K z)^T (d * (K z) + lambda z) and
<r, r>_K = r^T (K r), one kernel product K r per iteration, with K z and K delta carried by
the same recurrences as z and delta.  CG stops after max_cg iterations or once
sqrt(<r, r>_K) <= min(1/2, sqrt(||grad|| / ||grad_0||)) sqrt(<r_0, r_0>_K), then the step
backtracks t = 1, 1/2, ... until J(a + t delta) <= J(a) + 1e-4 t grad.delta (at most 30
halvings).  The outer loop stops when ||grad J|| <= tol ||grad J(0)|| or after max_newton
steps.  Products are the oracle's Table 4b double loop; everything else is FP64 numpy.
"""
from __future__ import annotations

import numpy as np

from . import pairwise_matvec

LOSSES = ("squared", "logistic", "sqhinge", "hinge")


def _sigma(x):
    # logistic function without overflow: 1 / (1 + exp(-x)) on either side of 0
    out = np.empty_like(x)
    pos = x >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-x[pos]))
    ex = np.exp(x[~pos])
    out[~pos] = ex / (1.0 + ex)
    return out


def loss_terms(loss, p, y):
    """(L, g, d): loss value, first and second derivative with respect to p."""
    p = np.asarray(p, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if loss == "squared":
        r = p - y
        return 0.5 * float(r @ r), r, np.ones_like(p)
    m = y * p
    if loss == "logistic":
        # log(1 + exp(-m)) = max(-m, 0) + log(1 + exp(-|m|))
        L = float(np.sum(np.maximum(-m, 0.0) + np.log1p(np.exp(-np.abs(m)))))
        s = _sigma(-m)
        return L, -y * s, s * (1.0 - s)
    h = np.maximum(0.0, 1.0 - m)
    if loss == "sqhinge":
        return 0.5 * float(h @ h), -y * h, (h > 0).astype(np.float64)
    if loss == "hinge":
        act = (h > 0).astype(np.float64)
        return float(np.sum(h)), -y * act, np.zeros_like(p)
    raise ValueError(loss)


def _K(kind, D, T, pairs, v):
    return pairwise_matvec(kind, D, T, pairs, pairs, v)


def objective(kind, D, T, pairs, y, a, lam, loss):
    """J(a) and its (sub)gradient K (g + lambda a) (Section 3 risk in dual coefficients)."""
    a = np.asarray(a, dtype=np.float64)
    p = _K(kind, D, T, pairs, a)
    L, g, _ = loss_terms(loss, p, y)
    J = L + 0.5 * lam * float(a @ p)
    grad = _K(kind, D, T, pairs, g + lam * a)
    return J, grad


def newton(kind, D, T, pairs, y, lam, loss, max_newton=20, max_cg=50, tol=1e-8):
    """Truncated Newton from a = 0 (see the module docstring).  Returns a dict with the
    solution a, Newton steps, total CG iterations, J and ||grad J|| at a, ||grad J(0)||."""
    if loss == "hinge":
        raise ValueError("the hinge loss has no Hessian; use its subgradient")
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    a = np.zeros(n)
    p = np.zeros(n)
    g0 = None
    steps = 0
    cg_total = 0
    while True:
        p = _K(kind, D, T, pairs, a)
        L, g, d = loss_terms(loss, p, y)
        J = L + 0.5 * lam * float(a @ p)
        grad = _K(kind, D, T, pairs, g + lam * a)
        gn = float(np.sqrt(grad @ grad))
        if g0 is None:
            g0 = gn
        if steps >= max_newton or gn <= tol * g0 or gn == 0.0:
            break
        eta = min(0.5, np.sqrt(gn / g0))
        x = np.zeros(n)
        Kx = np.zeros(n)
        r = -(g + lam * a)
        Kr = -grad
        z = r.copy()
        Kz = Kr.copy()
        rho = float(r @ Kr)
        rho0 = rho
        for _ in range(max_cg):
            Az = d * Kz + lam * z
            zAz = float(Kz @ Az)
            cg_total += 1
            if not (zAz > 0.0 and rho > 0.0):
                break
            alpha = rho / zAz
            x = x + alpha * z
            Kx = Kx + alpha * Kz
            r = r - alpha * Az
            Kr = _K(kind, D, T, pairs, r)
            rho_new = float(r @ Kr)
            if not rho_new > 0.0 or np.sqrt(rho_new) <= eta * np.sqrt(rho0):
                break
            beta = rho_new / rho
            z = r + beta * z
            Kz = Kr + beta * Kz
            rho = rho_new
        if not np.any(x):
            break
        slope = float(grad @ x)
        t = 1.0
        for _ in range(31):
            at = a + t * x
            Lt, _, _ = loss_terms(loss, p + t * Kx, y)
            Jt = Lt + 0.5 * lam * float(at @ (p + t * Kx))
            if Jt <= J + 1e-4 * t * slope:
                break
            t *= 0.5
        a = a + t * x
        steps += 1
    return dict(a=a, steps=steps, cg_iters=cg_total, J=J, gnorm=gn, gnorm0=g0)
