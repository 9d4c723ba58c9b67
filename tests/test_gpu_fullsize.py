"""Parity at the benchmark workloads' full sizes, in the launch configuration bench.py times.

The oracle cannot finish whole products at these sizes, so each test compares a seeded
sample of output rows: the oracle evaluates those rows one by one (every input pair, Table 4b
kernel function, FP64).  Tolerances as in test_gpu_parity (norm-wise, per kind and RHS).
"""
import numpy as np
import pytest

import oracle
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
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def ridge():
    return W.config2()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ridge_product_sampled_rows(gvt, ridge, prec):
    # m=2000, q=500, n=200000: the plan and kernels the ridge CG bench runs
    p = ridge
    dt = torch.float64 if prec == "f64" else torch.float32
    D, T = dev(p["D"], dt), dev(p["T"], dt)
    c, e = dev(p["c"]), dev(p["e"])
    v = np.random.default_rng(31).standard_normal(len(p["c"]))
    plan = gvt.gvt_plan_create("kronecker", D.shape, T.shape, (c, e), (c, e), flags=gvt.FLAG_SYMMETRIC_BASES)
    u = plan.execute(D, T, dev(v, dt))[0].double().cpu().numpy()
    plan.close()
    rows = np.random.default_rng(32).choice(len(p["c"]), 256, replace=False)
    ref = oracle.pairwise_matvec("kronecker", p["D"], p["T"], (p["c"], p["e"]), (p["c"], p["e"]), v, rows=rows)
    assert relerr(u[rows], ref) < (1e-10 if prec == "f64" else 1e-5)


def test_ridge_cg_true_residual_sampled(gvt, ridge):
    # the headline solve: its reported true residual, and the oracle's residual on sampled rows
    p = ridge
    A, iters, rel, rc = gvt.gvt_krr_cg("kronecker", dev(p["D"]), dev(p["T"]), (dev(p["c"]), dev(p["e"])),
                                       dev(p["y"]), [p["lam"]], max_iter=200, tol=1e-6, check_every=8)
    assert rc == 0 and rel[0] < 1e-6
    a = A[:, 0].cpu().numpy()
    rows = np.random.default_rng(33).choice(len(p["c"]), 256, replace=False)
    Ka = oracle.pairwise_matvec("kronecker", p["D"], p["T"], (p["c"], p["e"]), (p["c"], p["e"]), a, rows=rows)
    r_rows = p["y"][rows] - (Ka + p["lam"] * a[rows])
    # the residual on 256 of 200000 rows, scaled to the whole vector, is of the order the solver reports
    est = np.linalg.norm(r_rows) * np.sqrt(len(p["c"]) / len(rows)) / np.linalg.norm(p["y"])
    assert est < 10 * 1e-6


def test_fused_kinds_full_size_sampled(gvt):
    # symmetric + anti-symmetric + Cartesian + Poly2D, m=5000, n=1M unordered pairs, FP32
    kinds = ["symmetric", "antisymmetric", "cartesian", "poly2d"]
    p = W.config3()
    c, e = dev(p["c"]), dev(p["e"])
    D = dev(p["D"], torch.float32)
    plan = gvt.gvt_plan_create(kinds, D.shape, D.shape, (c, e), (c, e), flags=gvt.FLAG_SYMMETRIC_BASES)
    out = plan.execute(D, D, dev(p["v"], torch.float32)).double().cpu().numpy()
    plan.close()
    rows = np.random.default_rng(34).choice(len(p["c"]), 128, replace=False)
    for k, kind in enumerate(kinds):
        ref = oracle.pairwise_matvec(kind, p["D"], None, (p["c"], p["e"]), (p["c"], p["e"]), p["v"], rows=rows)
        assert relerr(out[k][rows], ref) < 1e-5, kind


@pytest.fixture(scope="module")
def complete():
    return W.config4()


@pytest.fixture(scope="module")
def complete_ref(complete):
    # 32 sampled entries of Umat by the oracle (each sums all 33.5M input pairs), and the
    # magnitude product |M||V||N|^T at those entries for the bf16x3 error bound
    p = complete
    m, q = p["m"], p["q"]
    rng = np.random.default_rng(35)
    ent = rng.choice(m * q, 32, replace=False)
    a_all = (np.arange(m * q) // q).astype(np.int32)
    b_all = (np.arange(m * q) % q).astype(np.int32)
    ref = oracle.pairwise_matvec("kronecker", p["D"], p["T"], (a_all, b_all), (a_all, b_all), p["V"].ravel(),
                                 rows=ent)
    ri, ci = ent // q, ent % q
    mag = np.einsum("ik,ik->i", np.abs(p["D"][ri]) @ np.abs(p["V"]), np.abs(p["T"][ci]))
    return ent, ref, mag


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6"])
def test_complete_data_full_size_sampled(gvt, complete, complete_ref, prec):
    # m=8192, q=4096: Umat = M Vmat N^T on matrix cores, 32 sampled entries against the oracle
    p = complete
    ent, ref, mag = complete_ref
    dt = torch.float64 if prec == "f64" else torch.float32
    pc = {"f64": gvt.F64, "f32": gvt.F32, "bf16x3": gvt.BF16X3, "bf16x6": gvt.BF16X6}[prec]
    U = gvt.gvt_dense_matvec(dev(p["D"], dt), dev(p["T"], dt), dev(p["V"], dt), prec=pc)
    got = U.reshape(-1)[torch.from_numpy(ent).cuda()].double().cpu().numpy()
    if prec == "bf16x3":
        # ~16 significant bits per operand: |dU| <= 4 * 2^-16 |M||V||N|^T
        assert np.linalg.norm(got - ref) <= 4 * 2.0 ** -16 * np.linalg.norm(mag)
    else:
        assert relerr(got, ref) < {"f64": 1e-10, "f32": 1e-5, "bf16x6": 1e-5}[prec]


def test_batched_full_size_problem_sample(gvt):
    # three problems of the 256-problem set (smallest, median, largest n) solved in one batch,
    # FP32 products: certified true residuals, and solutions against the oracle for the smallest
    shapes = W.config5_shapes()
    order = sorted(range(len(shapes)), key=lambda i: shapes[i][2])
    pick = [order[0], order[len(order) // 2], order[-1]]
    probs = [W.config5_problem(i, shapes[i]) for i in pick]
    dp = [dict(D=dev(q["D"]), T=dev(q["T"]), c=dev(q["c"]), e=dev(q["e"]), y=dev(q["y"])) for q in probs]
    lams = list(W.LAMBDA_GRID)
    A, iters, rel, rc = gvt.gvt_krr_cg_batched("kronecker", dp, lams, max_iter=200, tol=1e-6,
                                               matvec_prec=gvt.F32)
    assert rc in (0, 1)
    assert ((rel < 1e-6) | (iters == 200)).all()
    q = probs[0]
    A_or, it_or, _, rt_or = oracle.krr_cg("kronecker", q["D"], q["T"], (q["c"], q["e"]), q["y"], lams,
                                          max_iter=200, tol=1e-6)
    a = A[0].cpu().numpy()
    for l in range(len(lams)):
        if rt_or[l] < 1e-6 and rel[0, l] < 1e-6:
            assert relerr(a[:, l], A_or[:, l]) < 1e-4
