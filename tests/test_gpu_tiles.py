"""Dense tiles for dense-but-incomplete data: a single Kronecker term computed as
M Vmat N^T on matrix cores (v scattered into a zero grid, outputs gathered), against the
oracle's double loop (Theorem 1's product, the complete-data identity of Section 3)."""
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
    return (t.to(dtype) if dtype is not None else t).cuda()


def idx(x):
    return dev(np.asarray(x, dtype=np.int32))


def relerr(got, ref):
    got = np.asarray(got, np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, np.float64).reshape(len(ref), -1)
    return max(np.linalg.norm(got[:, r] - ref[:, r]) / np.linalg.norm(ref[:, r]) for r in range(ref.shape[1]))


TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-4}


def _run(gvt, p, prec, flags, nrhs_v):
    dt = torch.float64 if prec == "f64" else torch.float32
    pc = {"f64": gvt.F64, "f32": gvt.F32, "bf16x3": gvt.BF16X3, "bf16x6": gvt.BF16X6}[prec]
    D, T = dev(p["D"], dt), dev(p["T"], dt)
    plan = gvt.gvt_plan_create("kronecker", D.shape, T.shape, (idx(p["a"]), idx(p["b"])),
                               (idx(p["c"]), idx(p["e"])), flags=flags)
    u = plan.execute(D, T, dev(nrhs_v, dt), prec=pc)
    plan.close()
    return u.double().cpu().numpy().reshape(len(p["a"]), -1)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("order", ["A", "B"])
def test_tiles_match_oracle(gvt, prec, order):
    # 30% of a 150 x 130 grid, a separate output sample, duplicated input pairs, 3 RHS
    p = W.make_heterogeneous(101, 0, 150, 130, 5850, 8, n_out=3000)
    p["c"][:40] = p["c"][40:80]
    p["e"][:40] = p["e"][40:80]
    v = np.random.default_rng(102).standard_normal((len(p["c"]), 3))
    ref = oracle.pairwise_matvec("kronecker", p["D"], p["T"], (p["a"], p["b"]), (p["c"], p["e"]), v)
    fl = gvt.FLAG_DENSE_TILES | (gvt.FLAG_ORDER_A if order == "A" else gvt.FLAG_ORDER_B)
    u = _run(gvt, p, prec, fl, v)
    assert relerr(u, ref) < TOL[prec]
    if prec in ("f64", "f32"):
        g = _run(gvt, p, prec, gvt.FLAG_NO_DENSE_TILES, v)  # the gather path on the same plan shape
        assert relerr(g, ref) < TOL[prec]


def test_tiles_rectangular_prediction(gvt):
    # prediction for new objects: D is 90 x 60 (test x training drugs), T 70 x 50
    r = np.random.default_rng(103)
    Xd, Xt = r.standard_normal((90, 6)), r.standard_normal((70, 6))
    D = W.gaussian_kernel(Xd, Xd[:60])
    T = W.gaussian_kernel(Xt, Xt[:50])
    cells = r.choice(60 * 50, 1200, replace=False)
    c, e = (cells // 50).astype(np.int32), (cells % 50).astype(np.int32)
    a, b = r.integers(0, 90, 800).astype(np.int32), r.integers(0, 70, 800).astype(np.int32)
    v = r.standard_normal(1200)
    ref = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    p = dict(D=D, T=T, a=a, b=b, c=c, e=e)
    for prec in ("f64", "f32"):
        assert relerr(_run(gvt, p, prec, gvt.FLAG_DENSE_TILES, v), ref) < TOL[prec]


def test_tiles_cost_model_choices(gvt):
    # the ridge workload's skinny GEMMs (2000 x 500 outputs) lose to the gather path at 20%
    # density; a large grid at 50% density takes the tiles; bf16 forms always do
    p = W.config2()
    c, e = idx(p["c"]), idx(p["e"])
    pl = gvt.gvt_plan_create("kronecker", (2000, 2000), (500, 500), (c, e), (c, e))
    assert not gvt.gvt_plan_uses_tiles(pl, gvt.F64) and not gvt.gvt_plan_uses_tiles(pl, gvt.F32)
    assert gvt.gvt_plan_uses_tiles(pl, gvt.BF16X3)
    pl.close()
    r = np.random.default_rng(107)
    cells = r.choice(4096 * 2048, 4096 * 1024, replace=False)
    c2, e2 = idx(cells // 2048), idx(cells % 2048)
    pl = gvt.gvt_plan_create("kronecker", (4096, 4096), (2048, 2048), (c2, e2), (c2, e2))
    assert gvt.gvt_plan_uses_tiles(pl, gvt.F64) and gvt.gvt_plan_uses_tiles(pl, gvt.F32)
    pl.close()


def test_tiles_full_size_ridge_sampled(gvt):
    # m=2000, q=500, n=200000 (20%): the ridge workload's product through dense tiles
    p = W.config2()
    v = np.random.default_rng(104).standard_normal(len(p["c"]))
    rows = np.random.default_rng(105).choice(len(p["c"]), 256, replace=False)
    ref = oracle.pairwise_matvec("kronecker", p["D"], p["T"], (p["c"], p["e"]), (p["c"], p["e"]), v, rows=rows)
    for prec in ("f64", "f32", "bf16x6"):
        u = _run(gvt, p, prec, gvt.FLAG_DENSE_TILES | gvt.FLAG_SYMMETRIC_BASES, v)
        assert relerr(u[rows], ref) < TOL[prec], prec


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cg_with_tiles_products(gvt, monkeypatch, prec):
    # the ridge CG with its products on dense tiles: FP64 products against the oracle's CG;
    # FP32 products (FP64-certified) reach the same status and iterate as on the gather path
    p = W.make_heterogeneous(106, 0, 150, 120, 6000, 16, labels=True)
    args = ("kronecker", dev(p["D"]), dev(p["T"]), (idx(p["c"]), idx(p["e"])), dev(p["y"]), [0.3, 3.0])
    pc = gvt.F64 if prec == "f64" else gvt.F32
    monkeypatch.setenv("GVT_DENSE_TILES", "1")
    A, iters, rel, rc = gvt.gvt_krr_cg(*args, max_iter=400, tol=1e-6, matvec_prec=pc)
    monkeypatch.setenv("GVT_DENSE_TILES", "0")
    Ag, itg, relg, rcg = gvt.gvt_krr_cg(*args, max_iter=400, tol=1e-6, matvec_prec=pc)
    print(prec, "tiles", iters, rel, rc, "gather", itg, relg, rcg)
    assert rc == rcg == 0 and (rel < 1e-6).all()
    A, Ag = A.cpu().numpy(), Ag.cpu().numpy()
    # both solve the system to a 1e-6 residual over ~100 iterations: solutions agree to
    # about kappa * tol, not to rounding
    for l in range(2):
        assert np.linalg.norm(A[:, l] - Ag[:, l]) / np.linalg.norm(Ag[:, l]) < (1e-5 if prec == "f64" else 1e-4)
    if prec == "f64":
        A_or, it_or, _, rt_or = oracle.krr_cg("kronecker", p["D"], p["T"], (p["c"], p["e"]), p["y"], [0.3, 3.0],
                                              max_iter=400, tol=1e-6)
        for l in range(2):
            assert np.linalg.norm(A[:, l] - A_or[:, l]) / np.linalg.norm(A_or[:, l]) < 1e-5


# ------------------------------------------------------- plans of several terms
def _run_kinds(gvt, kinds, p, prec, flags, v):
    dt = torch.float64 if prec == "f64" else torch.float32
    pc = {"f64": gvt.F64, "f32": gvt.F32, "bf16x3": gvt.BF16X3, "bf16x6": gvt.BF16X6}[prec]
    D, T = dev(p["D"], dt), dev(p["T"], dt)
    plan = gvt.gvt_plan_create(kinds, D.shape, T.shape, (idx(p["a"]), idx(p["b"])),
                               (idx(p["c"]), idx(p["e"])), flags=flags)
    uses = gvt.gvt_plan_uses_tiles(plan, pc)
    u = plan.execute(D, T, dev(v, dt), prec=pc)  # (kinds, n_out[, rhs])
    plan.close()
    return u.double().cpu().numpy(), uses


HOM_KINDS = [["symmetric"], ["antisymmetric"], ["poly2d"], ["symmetric", "antisymmetric", "cartesian", "poly2d"]]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("kinds", HOM_KINDS, ids=["sym", "anti", "poly2d", "fused4"])
def test_multiterm_tiles_match_oracle(gvt, prec, kinds):
    # homogeneous kinds: both gather orders of the two-factor terms share one dense product
    # D Vmat D; one-factor (Poly2D) and match (Cartesian) terms stay on the gather path.
    # A separate output sample, duplicated input pairs, two RHS.
    p = W.make_homogeneous(108, 0, 160, 4000, 8, n_out=2500, kernel="gaussian")
    p["c"][:30] = p["c"][30:60]
    p["e"][:30] = p["e"][30:60]
    v = np.random.default_rng(109).standard_normal((len(p["c"]), 2))
    u, uses = _run_kinds(gvt, kinds, p, prec, gvt.FLAG_DENSE_TILES, v)
    assert uses == 1
    for k, kind in enumerate(kinds):
        ref = oracle.pairwise_matvec(kind, p["D"], None, (p["a"], p["b"]), (p["c"], p["e"]), v)
        err = relerr(u[k], ref)
        print(kind, prec, err)
        assert err < TOL[prec], (kind, prec, err)
        if prec == "f64":
            g, guse = _run_kinds(gvt, kinds, p, prec, gvt.FLAG_NO_DENSE_TILES, v)
            assert guse == 0 and relerr(g[k], ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_multiterm_tiles_heterogeneous(gvt, prec):
    # Kronecker + Poly2D + linear on a rectangular grid: one group D Vmat T^T serves the
    # Kronecker term and Poly2D's cross term; the one-factor terms run on the gather path
    kinds = ["kronecker", "poly2d", "linear"]
    p = W.make_heterogeneous(110, 0, 120, 90, 3000, 6, n_out=2000)
    v = np.random.default_rng(111).standard_normal(len(p["c"]))
    u, uses = _run_kinds(gvt, kinds, p, prec, gvt.FLAG_DENSE_TILES, v)
    assert uses == 1
    for k, kind in enumerate(kinds):
        ref = oracle.pairwise_matvec(kind, p["D"], p["T"], (p["a"], p["b"]), (p["c"], p["e"]), v)
        assert relerr(u[k], ref) < TOL[prec], (kind, prec)


def test_multiterm_tiles_not_for_degenerate_terms(gvt):
    # MLPK keys two of its two-factor terms by (c, c) and (e, e): no dense-tile form, so
    # its split-bf16 products are unsupported and FP64 runs the gather path
    p = W.make_homogeneous(112, 0, 60, 800, 6, kernel="gaussian")
    D = dev(p["D"])
    plan = gvt.gvt_plan_create(["mlpk"], D.shape, D.shape, (idx(p["a"]), idx(p["b"])),
                               (idx(p["c"]), idx(p["e"])), flags=gvt.FLAG_DENSE_TILES)
    assert gvt.gvt_plan_uses_tiles(plan, gvt.F64) == 0
    with pytest.raises(gvt.GvtError) as ei:
        plan.execute(D.float(), D.float(), dev(p["v"], torch.float32), prec=gvt.BF16X3)
    assert ei.value.code == -7
    plan.close()
