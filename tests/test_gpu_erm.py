"""Other losses on the same operator (Section 3's regularized risk; Section 7): the GPU's
objective, gradient and truncated Newton solver against the oracle's (tests/oracle erm)."""
import numpy as np
import pytest

import oracle
from oracle import erm
from paper_2009_01054_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gvt():
    import paper_2009_01054_amd as g

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.load_library()
    return g


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def idx(x):
    return dev(np.asarray(x, dtype=np.int32))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def _problem(kind, seed=0):
    if kind == "symmetric":
        p = W.make_homogeneous(91, seed, 40, 500, 4, kernel="gaussian")
        T = None
        r = np.random.default_rng([91, seed])
        score = p["X"][p["c"]] @ p["X"][p["e"]].T.diagonal() if False else (p["X"][p["c"]] * p["X"][p["e"]]).sum(1)
    else:
        p = W.make_heterogeneous(91, seed, 40, 35, 600, 4)
        T = p["T"]
        r = np.random.default_rng([91, seed])
        score = (p["Xd"][p["c"]] * p["Xt"][p["e"]]).sum(1)
    yb = np.where(score + 0.5 * r.standard_normal(len(score)) > 0, 1.0, -1.0)
    return p, T, yb


@pytest.mark.parametrize("loss", ["squared", "logistic", "sqhinge", "hinge"])
@pytest.mark.parametrize("kind", ["kronecker", "symmetric"])
def test_objective_and_gradient_match_oracle(gvt, kind, loss):
    p, T, yb = _problem(kind)
    a = 0.05 * np.random.default_rng(92).standard_normal(len(yb))
    lam = 0.2
    J_or, g_or = erm.objective(kind, p["D"], T, (p["c"], p["e"]), yb, a, lam, loss)
    J, g = gvt.gvt_erm_objective(kind, loss, dev(p["D"]), None if T is None else dev(T),
                                 (idx(p["c"]), idx(p["e"])), dev(yb), dev(a), lam)
    assert abs(J - J_or) <= 1e-11 * abs(J_or)
    assert rel(g.cpu().numpy(), g_or) < 1e-10
    J2, none = gvt.gvt_erm_objective(kind, loss, dev(p["D"]), None if T is None else dev(T),
                                     (idx(p["c"]), idx(p["e"])), dev(yb), dev(a), lam, grad=False)
    assert none is None and J2 == J


@pytest.mark.parametrize("loss", ["logistic", "sqhinge"])
def test_newton_fixed_steps_match_oracle(gvt, loss):
    # the same algorithm with the same constants: after 3 Newton steps of at most 8 CG
    # iterations the iterates agree up to rounding
    p, T, yb = _problem("kronecker", 1)
    lam = 0.1
    ref = erm.newton("kronecker", p["D"], T, (p["c"], p["e"]), yb, lam, loss, max_newton=3, max_cg=8, tol=0.0)
    res = gvt.gvt_erm_newton("kronecker", loss, dev(p["D"]), dev(T), (idx(p["c"]), idx(p["e"])), dev(yb), lam,
                             max_newton=3, max_cg=8, tol=0.0)
    assert res["steps"] == ref["steps"] == 3 and res["cg_iters"] == ref["cg_iters"]
    assert rel(res["a"].cpu().numpy(), ref["a"]) < 1e-8
    # J is not at its minimum after 3 steps: it moves with the iterate to first order
    assert abs(res["J"] - ref["J"]) <= 1e-8 * abs(ref["J"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,loss", [("kronecker", "logistic"), ("symmetric", "logistic"),
                                       ("kronecker", "sqhinge")])
def test_newton_converges_to_the_oracle_minimum(gvt, kind, loss, prec):
    p, T, yb = _problem(kind, 2)
    lam = 0.05
    ref = erm.newton(kind, p["D"], T, (p["c"], p["e"]), yb, lam, loss, max_newton=60, max_cg=200, tol=1e-10)
    tol = 1e-9 if prec == "f64" else 1e-5
    res = gvt.gvt_erm_newton(kind, loss, dev(p["D"]), None if T is None else dev(T), (idx(p["c"]), idx(p["e"])),
                             dev(yb), lam, max_newton=60, max_cg=200, tol=tol,
                             matvec_prec=gvt.F64 if prec == "f64" else gvt.F32)
    assert res["status"] == 0 and res["gnorm"] <= tol * res["gnorm0"]
    # the minimum value, and the predictions K a at the minimiser
    # FP32 products evaluate J itself to about 1e-7 relative per prediction
    assert abs(res["J"] - ref["J"]) <= (1e-10 if prec == "f64" else 1e-5) * abs(ref["J"])
    K_a = oracle.pairwise_matvec(kind, p["D"], T, (p["c"], p["e"]), (p["c"], p["e"]), res["a"].cpu().numpy())
    K_ref = oracle.pairwise_matvec(kind, p["D"], T, (p["c"], p["e"]), (p["c"], p["e"]), ref["a"])
    assert rel(K_a, K_ref) < (1e-5 if prec == "f64" else 1e-3)


def test_squared_loss_newton_is_the_ridge_solution(gvt):
    p = W.make_heterogeneous(93, 0, 30, 25, 400, 4, labels=True)
    D, T, inp, y = dev(p["D"]), dev(p["T"]), (idx(p["c"]), idx(p["e"])), dev(p["y"])
    res = gvt.gvt_erm_newton("kronecker", "squared", D, T, inp, y, 0.3, max_newton=40, max_cg=300, tol=1e-12)
    A, iters, rel_cg, rc = gvt.gvt_krr_cg("kronecker", D, T, inp, y, [0.3], max_iter=500, tol=1e-12)
    assert res["status"] == 0 and rc == 0
    assert rel(res["a"].cpu().numpy(), A[:, 0].cpu().numpy()) < 1e-8


def test_hinge_newton_is_unsupported(gvt):
    p, T, yb = _problem("kronecker")
    with pytest.raises(gvt.GvtError) as ei:
        gvt.gvt_erm_newton("kronecker", "hinge", dev(p["D"]), dev(T), (idx(p["c"]), idx(p["e"])), dev(yb), 0.1)
    assert ei.value.code == -7
