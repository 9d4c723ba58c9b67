"""Plans whose index work runs on the device (validation, unique counts, the
stable sorts into stage-1 key segments, output groupings and stage-2 tile
orders) against plans built on the host.

Both constructions sort stably, so they produce the same arrays and the
products agree bit for bit.  GVT_PLAN_DEVICE=0/1 forces the side; by default
index sets of 65536 pairs or more (output plus input) are planned on the device.
"""
import numpy as np
import pytest

import oracle
from paper_2009_01054_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HET = ["kronecker", "linear", "poly2d", "cartesian"]
HOM = ["symmetric", "antisymmetric", "ranking", "mlpk"]


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


def idx(x):
    return dev(np.asarray(x, dtype=np.int32))


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def both(monkeypatch, fn):
    """fn() with host-built and with device-built plans."""
    monkeypatch.setenv("GVT_PLAN_DEVICE", "0")
    h = fn()
    monkeypatch.setenv("GVT_PLAN_DEVICE", "1")
    d = fn()
    monkeypatch.delenv("GVT_PLAN_DEVICE")
    return h, d


@pytest.mark.parametrize("nrhs", [1, 3, 8])
@pytest.mark.parametrize("kind", HET + HOM)
def test_every_kind_bitwise(gvt, monkeypatch, kind, nrhs):
    if kind in HOM:
        p = W.make_homogeneous(93, nrhs, 41, 650, 5, n_out=321, kernel="gaussian", nrhs=nrhs)
        T = p["D"]
    else:
        p = W.make_heterogeneous(94, nrhs, 37, 29, 700, 6, n_out=333, nrhs=nrhs)
        T = p["T"]
    Dd, Td = dev(p["D"]), dev(T)
    pa, pb, pc, pe, v = idx(p["a"]), idx(p["b"]), idx(p["c"]), idx(p["e"]), dev(p["v"])
    h, d = both(monkeypatch, lambda: gvt.gvt_pairwise_matvec(
        [kind], Dd, Td, (pa, pb), (pc, pe), v, flags=gvt.FLAG_SYMMETRIC_BASES))
    assert torch.equal(h, d)
    ref = oracle.pairwise_matvec(kind, p["D"], None if kind in HOM else T, (p["a"], p["b"]),
                                 (p["c"], p["e"]), p["v"])
    got = d[0].cpu().numpy().reshape(len(ref), -1)
    for r in range(got.shape[1]):
        assert relerr(got[:, r], np.asarray(ref).reshape(len(ref), -1)[:, r]) < 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_kinds_several_tiles_bitwise(gvt, monkeypatch, prec):
    # 300 objects, 20000 training and 9000 output pairs: several tiles per
    # term in both stage-2 tile classes (2 and 8 RHS), match-term groupings
    kinds = ["symmetric", "antisymmetric", "cartesian", "poly2d"]
    p = W.make_homogeneous(95, 0, 300, 20000, 16, n_out=9000, kernel="linear", nrhs=8)
    dt = torch.float64 if prec == "f64" else torch.float32
    Dd = dev(p["D"], dt)
    pa, pb, pc, pe = idx(p["a"]), idx(p["b"]), idx(p["c"]), idx(p["e"])
    for nrhs in (2, 8):
        v = dev(p["v"][:, :nrhs], dt)
        h, d = both(monkeypatch, lambda: gvt.gvt_pairwise_matvec(
            kinds, Dd, Dd, (pa, pb), (pc, pe), v, flags=gvt.FLAG_SYMMETRIC_BASES))
        assert torch.equal(h, d), nrhs


@pytest.mark.parametrize("order", [0, 2, 4])
@pytest.mark.parametrize("kind", ["kronecker", "mlpk"])
def test_stage_orders_and_rectangular_bitwise(gvt, monkeypatch, kind, order):
    r = np.random.default_rng([6, order])
    if kind == "mlpk":
        p = W.make_homogeneous(96, 1, 30, 300, 4, n_out=150, kernel="gaussian")
        D = p["D"] + 0.05 * r.standard_normal(p["D"].shape)
        T = D
        a, b, c, e, v = p["a"], p["b"], p["c"], p["e"], p["v"]
    else:
        # two-sample: 60 x 40 and 45 x 30 bases, distinct output and input pairs
        Xd, Xt = r.standard_normal((60, 4)), r.standard_normal((45, 4))
        D = W.gaussian_kernel(Xd, Xd[:40])
        T = W.gaussian_kernel(Xt, Xt[:30])
        c, e = W.sample_grid_pairs(r, 40, 30, 500)
        a, b = W.sample_grid_pairs(r, 60, 45, 800)
        v = r.standard_normal(500)
    Dd, Td = dev(D), dev(T)
    args = ((idx(a), idx(b)), (idx(c), idx(e)), dev(v))
    h, d = both(monkeypatch, lambda: gvt.gvt_pairwise_matvec([kind], Dd, Td, *args, flags=order))
    assert torch.equal(h, d)
    ref = oracle.pairwise_matvec(kind, D, None if kind == "mlpk" else T, (a, b), (c, e), v)
    assert relerr(d[0].cpu().numpy(), ref) < 1e-10


def test_duplicates_bitwise(gvt, monkeypatch):
    r = np.random.default_rng(14)
    m = 9
    D = W.gaussian_kernel(r.standard_normal((m, 3)))
    c = r.integers(0, m, 400).astype(np.int32)
    e = r.integers(0, m, 400).astype(np.int32)
    c[:50] = 3
    e[:50] = 3
    a = r.integers(0, m, 250).astype(np.int32)
    b = r.integers(0, m, 250).astype(np.int32)
    v = r.standard_normal(400)
    Dd = dev(D)
    for kind in ["kronecker", "cartesian", "mlpk"]:
        h, d = both(monkeypatch, lambda: gvt.gvt_pairwise_matvec(
            [kind], Dd, Dd, (idx(a), idx(b)), (idx(c), idx(e)), dev(v), flags=gvt.FLAG_SYMMETRIC_BASES))
        assert torch.equal(h, d), kind
        ref = oracle.pairwise_matvec(kind, D, D, (a, b), (c, e), v)
        assert relerr(d[0].cpu().numpy(), ref) < 1e-10, kind


def test_wide_key_range(gvt, monkeypatch):
    # 70000 x 70000 index ranges: the packed (key, other) sort key needs 34 bits
    r = np.random.default_rng(15)
    ncol = 70000
    D = r.standard_normal((5, ncol))
    T = r.standard_normal((4, ncol))
    c = r.integers(0, ncol, 3000).astype(np.int32)
    e = r.integers(0, ncol, 3000).astype(np.int32)
    c[:7] = ncol - 1  # the top of both ranges
    e[:7] = ncol - 1
    a = r.integers(0, 5, 50).astype(np.int32)
    b = r.integers(0, 4, 50).astype(np.int32)
    v = r.standard_normal(3000)
    Dd, Td = dev(D), dev(T)
    h, d = both(monkeypatch, lambda: gvt.gvt_matvec(Dd, Td, (idx(a), idx(b)), (idx(c), idx(e)), dev(v)))
    assert torch.equal(h, d)
    ref = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    assert relerr(d.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 300001])
def test_own_sort_matches_library_sort(gvt, monkeypatch, n):
    # the plan's stable radix sort (one to three passes of up to 10-bit digits, tiles of
    # 2048 pairs, a ragged last tile) against the library's radix sort on device-built
    # plans: a stable sort's order is unique, so the products agree bit for bit
    r = np.random.default_rng([16, n])
    m, q = 1500, 900
    D = W.gaussian_kernel(r.standard_normal((m, 3)))
    T = W.gaussian_kernel(r.standard_normal((q, 3)))
    c = r.integers(0, m, n).astype(np.int32)
    e = r.integers(0, q, n).astype(np.int32)
    a = r.integers(0, m, 5000).astype(np.int32)
    b = r.integers(0, q, 5000).astype(np.int32)
    v = r.standard_normal((n, 2))
    Dd, Td = dev(D), dev(T)
    monkeypatch.setenv("GVT_PLAN_DEVICE", "1")
    res = []
    for lib in ("1", "0"):
        monkeypatch.setenv("GVT_PLAN_LIBRARY_SORT", lib)
        res.append(gvt.gvt_matvec(Dd, Td, (idx(a), idx(b)), (idx(c), idx(e)), dev(v)))
    assert torch.equal(res[0], res[1])
    ref = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    assert relerr(res[1].cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("ncol", [1500, 70000])
def test_own_sort_matches_library_sort_at_scale(gvt, monkeypatch, ncol):
    # 4 000 037 pairs (3 907 tiles, a ragged last one): 21-bit keys in three passes over a
    # 1500 x 900 grid, and 34-bit keys in four passes over 70000 x 70000 index ranges;
    # products of device-built plans agree bit for bit with either sort
    r = np.random.default_rng([17, ncol])
    n = 4_000_037
    rows_d, rows_t = (1500, 900) if ncol == 1500 else (5, 4)
    cols_t = 900 if ncol == 1500 else ncol
    D = r.standard_normal((rows_d, ncol))
    T = r.standard_normal((rows_t, cols_t))
    c = r.integers(0, ncol, n).astype(np.int32)
    e = r.integers(0, cols_t, n).astype(np.int32)
    a = r.integers(0, rows_d, 3000).astype(np.int32)
    b = r.integers(0, rows_t, 3000).astype(np.int32)
    v = r.standard_normal(n)
    Dd, Td = dev(D), dev(T)
    monkeypatch.setenv("GVT_PLAN_DEVICE", "1")
    res = []
    for lib in ("1", "0"):
        monkeypatch.setenv("GVT_PLAN_LIBRARY_SORT", lib)
        res.append(gvt.gvt_matvec(Dd, Td, (idx(a), idx(b)), (idx(c), idx(e)), dev(v)))
    assert torch.equal(res[0], res[1])


def test_index_errors_on_device(gvt, monkeypatch):
    monkeypatch.setenv("GVT_PLAN_DEVICE", "1")
    D = dev(np.eye(5)); T = dev(np.eye(4))
    a = idx([0, 1, 2]); b = idx([0, 3, 4])  # b[2] = 4 is outside T's 4 rows
    with pytest.raises(gvt.GvtError) as ei:
        gvt.gvt_matvec(D, T, (a, b), (a, idx([0, 1, 2])), dev(np.ones(3)))
    assert ei.value.code == -2 and "out_b[2] = 4" in str(ei.value)
    with pytest.raises(gvt.GvtError) as ei:
        gvt.gvt_matvec(D, T, (a, idx([0, 1, 3])), (idx([0, -1, 2]), idx([0, 1, 2])), dev(np.ones(3)))
    assert ei.value.code == -2 and "in_c[1] = -1" in str(ei.value)


def test_empty_sets_on_device(gvt, monkeypatch):
    monkeypatch.setenv("GVT_PLAN_DEVICE", "1")
    D = dev(np.eye(5)); T = dev(np.eye(4))
    z = idx(np.zeros(0))
    a = idx([0, 1, 2]); b = idx([1, 2, 3])
    u = gvt.gvt_matvec(D, T, (a, b), (z, z), dev(np.zeros(0)))
    assert u.shape == (3,) and torch.count_nonzero(u) == 0
    u = gvt.gvt_matvec(D, T, (z, z), (a, b), dev(np.ones(3)))
    assert u.numel() == 0


def test_complete_data_detected_on_device(gvt, monkeypatch):
    r = np.random.default_rng(16)
    m, q = 24, 20
    D = W.gaussian_kernel(r.standard_normal((m, 3)))
    T = W.gaussian_kernel(r.standard_normal((q, 3)))
    a = np.repeat(np.arange(m), q).astype(np.int32)
    b = np.tile(np.arange(q), m).astype(np.int32)
    v = r.standard_normal(m * q)
    Dd, Td = dev(D), dev(T)
    h, d = both(monkeypatch, lambda: gvt.gvt_matvec(Dd, Td, (idx(a), idx(b)), (idx(a), idx(b)), dev(v)))
    assert torch.equal(h, d)
    assert relerr(d.cpu().numpy(), (D @ v.reshape(m, q) @ T.T).ravel()) < 1e-12


def test_cg_bitwise(gvt, monkeypatch):
    p = W.make_heterogeneous(97, 0, 60, 45, 1500, 6, labels=True)
    lam = [1e-2, 1e-1, 1.0]
    args = ("kronecker", dev(p["D"]), dev(p["T"]), (idx(p["c"]), idx(p["e"])), dev(p["y"]), lam)
    (Ah, ih, rh, ch), (Ad, i_d, rd, cd) = both(monkeypatch, lambda: gvt.gvt_krr_cg(*args, max_iter=200,
                                                                                     tol=1e-6))
    assert ch == cd and torch.equal(Ah, Ad) and (ih == i_d).all() and (rh == rd).all()


def test_cg_batched_bitwise(gvt, monkeypatch):
    probs = []
    for i, (m, q, n) in enumerate([(30, 20, 300), (50, 35, 900), (12, 40, 200)]):
        pr = W.make_heterogeneous(98, i, m, q, n, 6, labels=True)
        probs.append(dict(D=dev(pr["D"]), T=dev(pr["T"]), c=idx(pr["c"]), e=idx(pr["e"]), y=dev(pr["y"])))
    lam = [1e-3, 1e-1, 10.0]
    (Ah, ih, rh, ch), (Ad, i_d, rd, cd) = both(monkeypatch, lambda: gvt.gvt_krr_cg_batched(
        "kronecker", probs, lam, max_iter=200, tol=1e-6))
    assert ch == cd and (ih == i_d).all() and (rh == rd).all()
    for x, y in zip(Ah, Ad):
        assert torch.equal(x, y)
