"""Pins for the CPU oracle against what the paper and mathematics fix (no GPU).

Each test checks the oracle's Table 4b double loop against an independent
form: the printed operator example, explicitly formed Kronecker products and
Corollary 1 operators, Table 4a feature maps, closed forms, a library GEMM on
complete data, kernel invariants, and a dense LAPACK solve for the ridge CG.
"""
import os

import numpy as np
import pytest

import oracle
from tests import operators as ops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HET = ["kronecker", "linear", "poly2d", "cartesian"]
HOM = ["symmetric", "antisymmetric", "ranking", "mlpk"]


def _rng(s):
    return np.random.default_rng([7, s])


def _tiny_het(seed, m=4, q=3, n=17, n_out=11, dup=True):
    r = _rng(seed)
    D = r.standard_normal((m, m)); D = D @ D.T
    T = r.standard_normal((q, q)); T = T @ T.T
    c = r.integers(0, m, n).astype(np.int32)
    e = r.integers(0, q, n).astype(np.int32)
    if dup:
        c[1], e[1] = c[0], e[0]  # a duplicated pair
    a = r.integers(0, m, n_out).astype(np.int32)
    b = r.integers(0, q, n_out).astype(np.int32)
    v = r.standard_normal(n)
    return D, T, (a, b), (c, e), v


def _tiny_hom(seed, m=5, n=19, n_out=13):
    r = _rng(100 + seed)
    X = r.standard_normal((m, 3))
    D = X @ X.T + 0.1 * np.eye(m)
    c = r.integers(0, m, n).astype(np.int32)
    e = r.integers(0, m, n).astype(np.int32)
    c[1], e[1] = c[0], e[0]
    a = r.integers(0, m, n_out).astype(np.int32)
    b = r.integers(0, m, n_out).astype(np.int32)
    v = r.standard_normal(n)
    return D, (a, b), (c, e), v


# ---------------------------------------------------------- Definition 1 example
def test_printed_commutation_and_unification():
    P = np.loadtxt(os.path.join(GOLDEN, "commutation_P_D3_T2.txt"))
    Q = np.loadtxt(os.path.join(GOLDEN, "unification_Q_D3_T2.txt"))
    assert np.array_equal(ops.commutation(3, 2), P)
    assert np.array_equal(ops.unification(3, 2), Q)


def test_lemma_identities():
    r = _rng(1)
    D = r.standard_normal((3, 3)); T = r.standard_normal((2, 2))
    P = np.loadtxt(os.path.join(GOLDEN, "commutation_P_D3_T2.txt"))
    Q = np.loadtxt(os.path.join(GOLDEN, "unification_Q_D3_T2.txt"))
    assert np.allclose(P @ P.T, np.eye(6)) and np.allclose(P.T @ P, np.eye(6))
    assert np.allclose(P @ np.kron(D, T), np.kron(T, D) @ P)
    assert np.allclose(P @ np.kron(D, T) @ P.T, np.kron(T, D))
    # Q (D x D) Q^T = D^{o2} x 1 (Lemma, with Q mapping D x T -> D x D)
    assert np.allclose(Q @ np.kron(D, D) @ Q.T, np.kron(D * D, np.ones((2, 2))))
    Ph = ops.commutation(3, 3)
    assert np.array_equal(Ph, Ph.T)
    assert np.allclose(Ph @ np.kron(D, D) @ Ph, np.kron(D, D))


def test_sampling_operator_rules():
    """R(d,t) P = R(t,d) and R(d,t) Q = R(d,d) (proof of Corollary 1)."""
    d = np.array([0, 2, 1, 2]); t = np.array([1, 0, 1, 1])
    R = ops.sampling_operator(d, t, 3, 2)
    assert np.array_equal(R @ ops.commutation(3, 2).T, ops.sampling_operator(t, d, 2, 3))
    assert np.array_equal(R @ ops.unification(3, 2), ops.sampling_operator(d, d, 3, 3))


# -------------------------------------------------------------- core GVT (Kronecker)
@pytest.mark.parametrize("seed", range(4))
def test_kronecker_vs_explicit_kron(seed):
    D, T, (a, b), (c, e), v = _tiny_het(seed)
    Rb = ops.sampling_operator(a, b, *D.shape[:1], *T.shape[:1])
    R = ops.sampling_operator(c, e, D.shape[0], T.shape[0])
    ref = Rb @ np.kron(D, T) @ R.T @ v
    got = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_kronecker_rectangular_prediction():
    """Two-sample product with rectangular bases (test objects x training objects)."""
    r = _rng(9)
    Xd, Xt = r.standard_normal((7, 2)), r.standard_normal((5, 2))
    D = Xd @ Xd[:4].T  # 7 test drugs x 4 training drugs
    T = Xt @ Xt[:3].T  # 5 test targets x 3 training targets
    c = r.integers(0, 4, 12).astype(np.int32); e = r.integers(0, 3, 12).astype(np.int32)
    a = r.integers(0, 7, 9).astype(np.int32); b = r.integers(0, 5, 9).astype(np.int32)
    v = r.standard_normal(12)
    ref = np.array([sum(D[a[i], c[j]] * T[b[i], e[j]] * v[j] for j in range(12)) for i in range(9)])
    # via explicit Kronecker of the rectangular bases
    K = np.kron(D, T)
    ref2 = K[a * 5 + b][:, c * 3 + e] @ v
    got = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    np.testing.assert_allclose(got, ref, rtol=1e-13)
    np.testing.assert_allclose(got, ref2, rtol=1e-13)


def test_complete_data_is_library_gemm():
    """All pairs in natural order: u.reshape(m, q) = D V T^T (host BLAS)."""
    r = _rng(3)
    m, q = 6, 5
    D = r.standard_normal((m, m)); T = r.standard_normal((q, q))
    V = r.standard_normal((m, q))
    idx = np.arange(m * q)
    a, b = (idx // q).astype(np.int32), (idx % q).astype(np.int32)
    got = oracle.pairwise_matvec("kronecker", D, T, (a, b), (a, b), V.ravel())
    np.testing.assert_allclose(got.reshape(m, q), D @ V @ T.T, rtol=1e-12, atol=1e-12)


def test_closed_forms():
    r = _rng(4)
    m, q, n = 5, 4, 12
    idx = r.choice(m * q, n, replace=False)
    c, e = (idx // q).astype(np.int32), (idx % q).astype(np.int32)
    v = r.standard_normal(n)
    # identity bases, distinct pairs, outputs = inputs -> u = v exactly
    u = oracle.pairwise_matvec("kronecker", np.eye(m), np.eye(q), (c, e), (c, e), v)
    assert np.array_equal(u, v)
    # N = all-ones -> u_i = (M s)[a_i], s = per-drug segment sums
    M = r.standard_normal((m, m))
    s = np.bincount(c, weights=v, minlength=m)
    u = oracle.pairwise_matvec("kronecker", M, np.ones((q, q)), (c, e), (c, e), v)
    np.testing.assert_allclose(u, (M @ s)[c], rtol=1e-12, atol=1e-12)
    # rank-one bases -> u_i = al[a_i] be[b_i] sum_j al[c_j] be[e_j] v_j
    al, be = r.standard_normal(m), r.standard_normal(q)
    u = oracle.pairwise_matvec("kronecker", np.outer(al, al), np.outer(be, be), (c, e), (c, e), v)
    np.testing.assert_allclose(u, al[c] * be[e] * np.sum(al[c] * be[e] * v), rtol=1e-12, atol=1e-12)


def test_commutation_swap():
    """GVT(M, N; a, b; c, e) = GVT(N, M; b, a; e, c) (Lemma, P (D x T) P^T = T x D)."""
    D, T, (a, b), (c, e), v = _tiny_het(5)
    u1 = oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)
    u2 = oracle.pairwise_matvec("kronecker", T, D, (b, a), (e, c), v)
    np.testing.assert_allclose(u1, u2, rtol=1e-13)


# --------------------------------------------------- every kind vs Corollary 1
@pytest.mark.parametrize("kind", HET)
@pytest.mark.parametrize("seed", range(3))
def test_heterogeneous_kinds_vs_corollary1(kind, seed):
    D, T, (a, b), (c, e), v = _tiny_het(seed)
    m, q = D.shape[0], T.shape[0]
    Kop = ops.corollary1_operator(kind, D, T)
    ref = ops.sampling_operator(a, b, m, q) @ Kop @ ops.sampling_operator(c, e, m, q).T @ v
    got = oracle.pairwise_matvec(kind, D, T, (a, b), (c, e), v)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("kind", HOM)
@pytest.mark.parametrize("seed", range(3))
def test_homogeneous_kinds_vs_corollary1(kind, seed):
    D, (a, b), (c, e), v = _tiny_hom(seed)
    m = D.shape[0]
    Kop = ops.corollary1_operator(kind, D)
    ref = ops.sampling_operator(a, b, m, m) @ Kop @ ops.sampling_operator(c, e, m, m).T @ v
    got = oracle.pairwise_matvec(kind, D, None, (a, b), (c, e), v)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1, np.abs(ref).max()))


def test_printed_antisymmetric_operator_has_opposite_sign():
    """The operator printed in Corollary 1, (P - I)(D x D), is the negative of the
    Table 4b function; the oracle follows the function (reading (I - P))."""
    D, (a, b), (c, e), v = _tiny_hom(7)
    m = D.shape[0]
    Kp = ops.corollary1_operator("antisymmetric", D, antisym_as_printed=True)
    ref_printed = ops.sampling_operator(a, b, m, m) @ Kp @ ops.sampling_operator(c, e, m, m).T @ v
    got = oracle.pairwise_matvec("antisymmetric", D, None, (a, b), (c, e), v)
    np.testing.assert_allclose(got, -ref_printed, rtol=1e-12, atol=1e-12)
    # the printed form is negative semidefinite on the full domain
    assert np.linalg.eigvalsh(0.5 * (Kp + Kp.T)).max() < 1e-9


def test_mlpk_needs_the_transpose():
    D, (a, b), (c, e), v = _tiny_hom(8)
    m = D.shape[0]
    Kbad = ops.corollary1_operator("mlpk", D, mlpk_without_transpose=True)
    Kgood = ops.corollary1_operator("mlpk", D)
    Kfun = oracle.kernel_matrix("mlpk", D, None, (np.repeat(np.arange(m), m), np.tile(np.arange(m), m)),
                                (np.repeat(np.arange(m), m), np.tile(np.arange(m), m)))
    np.testing.assert_allclose(Kgood, Kfun, rtol=1e-12, atol=1e-12)
    assert not np.allclose(Kbad, Kfun)


# ------------------------------------------------------------- Table 4a feature maps
@pytest.mark.parametrize("kind", HET + HOM)
def test_feature_maps_linear_bases(kind):
    r = _rng(11)
    hom = kind in HOM
    Xd = r.standard_normal((5, 3))
    Xt = None if hom else r.standard_normal((4, 2))
    D = Xd @ Xd.T
    T = None if hom else Xt @ Xt.T
    q = 5 if hom else 4
    n, n_out = 14, 9
    c = r.integers(0, 5, n).astype(np.int32); e = r.integers(0, q, n).astype(np.int32)
    a = r.integers(0, 5, n_out).astype(np.int32); b = r.integers(0, q, n_out).astype(np.int32)
    Phi_out = ops.feature_map(kind, Xd, Xt, a, b)
    Phi_in = ops.feature_map(kind, Xd, Xt, c, e)
    K_map = Phi_out @ Phi_in.T
    K = oracle.kernel_matrix(kind, D, T, (a, b), (c, e))
    np.testing.assert_allclose(K, K_map, rtol=1e-12, atol=1e-12)


def test_elementwise_square_relations():
    D, T, out, inp, _ = _tiny_het(12)
    np.testing.assert_allclose(oracle.kernel_matrix("poly2d", D, T, out, inp),
                               oracle.kernel_matrix("linear", D, T, out, inp) ** 2, rtol=1e-12)
    Dh, outh, inph, _ = _tiny_hom(12)
    np.testing.assert_allclose(oracle.kernel_matrix("mlpk", Dh, None, outh, inph),
                               oracle.kernel_matrix("ranking", Dh, None, outh, inph) ** 2, rtol=1e-12)


# ------------------------------------------------------------------ invariants
def test_symmetric_antisymmetric_invariants():
    D, (a, b), (c, e), v = _tiny_hom(13)
    us = oracle.pairwise_matvec("symmetric", D, None, (a, b), (c, e), v)
    ua = oracle.pairwise_matvec("antisymmetric", D, None, (a, b), (c, e), v)
    np.testing.assert_allclose(oracle.pairwise_matvec("symmetric", D, None, (b, a), (c, e), v), us, rtol=1e-12)
    np.testing.assert_allclose(oracle.pairwise_matvec("symmetric", D, None, (a, b), (e, c), v), us, rtol=1e-12)
    np.testing.assert_allclose(oracle.pairwise_matvec("antisymmetric", D, None, (b, a), (c, e), v), -ua, rtol=1e-12)
    # swapping input pair j is the same as negating v_j
    c2, e2, v2 = c.copy(), e.copy(), v.copy()
    c2[3], e2[3] = e[3], c[3]
    v2[3] = -v[3]
    np.testing.assert_allclose(oracle.pairwise_matvec("antisymmetric", D, None, (a, b), (c2, e2), v),
                               oracle.pairwise_matvec("antisymmetric", D, None, (a, b), (c, e), v2), rtol=1e-12, atol=1e-12)
    # K_sym + K_anti = 2 GVT(D,D;(a,b),(c,e)); K_sym - K_anti = 2 GVT(D,D;(b,a),(c,e))
    gA = oracle.pairwise_matvec("kronecker", D, D, (a, b), (c, e), v)
    gB = oracle.pairwise_matvec("kronecker", D, D, (b, a), (c, e), v)
    np.testing.assert_allclose(us + ua, 2 * gA, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(us - ua, 2 * gB, rtol=1e-12, atol=1e-12)
    ur = oracle.pairwise_matvec("ranking", D, None, (b, a), (c, e), v)
    np.testing.assert_allclose(ur, -oracle.pairwise_matvec("ranking", D, None, (a, b), (c, e), v), rtol=1e-12, atol=1e-12)
    um = oracle.pairwise_matvec("mlpk", D, None, (b, a), (c, e), v)
    np.testing.assert_allclose(um, oracle.pairwise_matvec("mlpk", D, None, (a, b), (c, e), v), rtol=1e-12)


@pytest.mark.parametrize("kind", HET + HOM)
def test_psd_selfadjoint_linear(kind):
    r = _rng(14)
    if kind in HOM:
        D, _, (c, e), _ = _tiny_hom(14, n=15)
        T = None
    else:
        D, T, _, (c, e), _ = _tiny_het(14, n=15)
    v, w = r.standard_normal(15), r.standard_normal(15)
    Kv = oracle.pairwise_matvec(kind, D, T, (c, e), (c, e), v)
    Kw = oracle.pairwise_matvec(kind, D, T, (c, e), (c, e), w)
    assert v @ Kv >= -1e-10 * max(1.0, np.abs(Kv).max())
    np.testing.assert_allclose(v @ Kw, w @ Kv, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(oracle.pairwise_matvec(kind, D, T, (c, e), (c, e), 2 * v - 3 * w),
                               2 * Kv - 3 * Kw, rtol=1e-11, atol=1e-11)


# --------------------------------------------------------- modes and determinism
def test_row_sampling_and_thread_independence():
    D, T, (a, b), (c, e), v = _tiny_het(15, m=9, q=7, n=300, n_out=200)
    V = np.stack([v, -2 * v + 1], axis=1)
    full1 = oracle.pairwise_matvec("poly2d", D, T, (a, b), (c, e), V, nthreads=1)
    full4 = oracle.pairwise_matvec("poly2d", D, T, (a, b), (c, e), V, nthreads=4)
    assert np.array_equal(full1, full4)
    rows = np.array([5, 0, 199, 42])
    part = oracle.pairwise_matvec("poly2d", D, T, (a, b), (c, e), V, rows=rows)
    assert np.array_equal(part, full1[rows])


def test_bad_index_rejected():
    D, T, (a, b), (c, e), v = _tiny_het(16)
    c = c.copy(); c[0] = D.shape[1]
    with pytest.raises(ValueError):
        oracle.pairwise_matvec("kronecker", D, T, (a, b), (c, e), v)


# ------------------------------------------------------------------------ ridge CG
@pytest.mark.parametrize("kind", ["kronecker", "symmetric", "poly2d"])
def test_cg_matches_dense_solve(kind):
    r = _rng(17)
    if kind == "symmetric":
        m, n = 12, 60
        X = r.standard_normal((m, 4))
        D = np.exp(-((X[:, None] - X[None]) ** 2).sum(-1) / 8)
        T = None
        c = r.integers(0, m, n).astype(np.int32); e = r.integers(0, m, n).astype(np.int32)
    else:
        m, q, n = 10, 8, 60
        Xd, Xt = r.standard_normal((m, 4)), r.standard_normal((q, 4))
        D = np.exp(-((Xd[:, None] - Xd[None]) ** 2).sum(-1) / 8)
        T = np.exp(-((Xt[:, None] - Xt[None]) ** 2).sum(-1) / 8)
        idx = r.choice(m * q, n, replace=False)
        c, e = (idx // q).astype(np.int32), (idx % q).astype(np.int32)
    y = r.standard_normal(n)
    lams = np.array([1e-1, 1.0, 10.0])
    A, iters, rr, rt = oracle.krr_cg(kind, D, T, (c, e), y, lams, max_iter=500, tol=1e-10)
    K = oracle.kernel_matrix(kind, D, T, (c, e), (c, e))
    for l, lam in enumerate(lams):
        ref = np.linalg.solve(K + lam * np.eye(n), y)
        cond = np.linalg.cond(K + lam * np.eye(n))
        assert np.linalg.norm(A[:, l] - ref) / np.linalg.norm(ref) < 10 * cond * 1e-10
        assert rt[l] < 1e-9 and iters[l] <= 500


# ------------------------------------------------- multi-RHS columns and strides
def _raw_matvec(kind, D, T, out_pairs, in_pairs, V, ldv, ldu, nev):
    """Call the C oracle directly with explicit column strides (padding filled with NaN)."""
    import ctypes

    lib = oracle._load()
    D = np.ascontiguousarray(D, dtype=np.float64)
    T = D if T is None else np.ascontiguousarray(T, dtype=np.float64)
    a, b = (np.ascontiguousarray(x, dtype=np.int32) for x in out_pairs)
    c, e = (np.ascontiguousarray(x, dtype=np.int32) for x in in_pairs)
    n, nrhs = V.shape
    vbuf = np.full(ldv * nrhs, np.nan)
    for s in range(nrhs):
        vbuf[s * ldv: s * ldv + n] = V[:, s]
    ubuf = np.full(ldu * nrhs, -7.5)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = lib.oracle_pairwise_matvec(
        oracle.KINDS[kind], p(D), D.shape[0], D.shape[1], D.shape[1], p(T), T.shape[0], T.shape[1],
        T.shape[1], p(a), p(b), len(a), None, 0, p(c), p(e), n, p(vbuf), nrhs, ldv, p(ubuf), ldu, 0)
    assert rc == 0
    return ubuf


@pytest.mark.parametrize("kind", HET + HOM)
def test_multi_rhs_columns_with_padded_strides(kind):
    """Each column of an n x 3 product with ldv > n and ldu > n_out equals the one-column
    product bit for bit and the explicit R(a,b) K R(c,e)^T v of that column; the padding
    of U is never written and the NaN padding of V is never read."""
    if kind in HOM:
        D, (a, b), (c, e), _ = _tiny_hom(21)
        T = None
        K = ops.corollary1_operator(kind, D)
        nd = nt = D.shape[0]
    else:
        D, T, (a, b), (c, e), _ = _tiny_het(21)
        K = ops.corollary1_operator(kind, D, T)
        nd, nt = D.shape[0], T.shape[0]
    r = _rng(22)
    n, n_out = len(c), len(a)
    V = r.standard_normal((n, 3))
    V[:, 2] = -3.0 * V[:, 0] + V[:, 1]
    ldv, ldu = n + 5, n_out + 3
    ubuf = _raw_matvec(kind, D, T, (a, b), (c, e), V, ldv, ldu, n_out)
    Rb = ops.sampling_operator(a, b, nd, nt)
    R = ops.sampling_operator(c, e, nd, nt)
    for s in range(3):
        col = ubuf[s * ldu: s * ldu + n_out]
        one = oracle.pairwise_matvec(kind, D, T, (a, b), (c, e), V[:, s])
        assert np.array_equal(col, one)
        ref = Rb @ K @ R.T @ V[:, s]
        np.testing.assert_allclose(col, ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))
        assert np.all(ubuf[s * ldu + n_out: (s + 1) * ldu] == -7.5)


# ------------------------------------ Cartesian kernel on two samples of objects
def _cartesian_feature_kernel(Xd, Xt, ud_out, ut_out, ud_in, ut_in):
    """Table 4a Cartesian feature map over a shared universe of objects: a pair of
    universe objects (d, t) maps to (x_d (x) e_t, e_d (x) x_t), e the universe one-hot."""
    nd, nt = Xd.shape[0], Xt.shape[0]

    def phi(ud, ut):
        f1 = np.einsum("ni,nj->nij", Xd[ud], np.eye(nt)[ut]).reshape(len(ud), -1)
        f2 = np.einsum("ni,nj->nij", np.eye(nd)[ud], Xt[ut]).reshape(len(ud), -1)
        return np.concatenate([f1, f2], axis=1)

    return phi(ud_out, ut_out) @ phi(ud_in, ut_in).T


def test_cartesian_rectangular_bases_shared_objects():
    """Cartesian delta on rectangular two-sample bases (reading R22): row r and column c
    of a base matrix are the same object iff r == c, so the prediction sample lists the
    training objects first, in training order, then objects absent from training.
    Checked against the Table 4a feature map over the object universe, with training
    objects that are a permuted subset of the universe and prediction objects that extend
    them; a prediction sample that permutes the shared objects breaks the correspondence."""
    r = _rng(23)
    Xd, Xt = r.standard_normal((9, 3)), r.standard_normal((8, 2))
    tr_d = np.array([6, 1, 4, 0])            # training drugs (universe ids, permuted)
    tr_t = np.array([5, 2, 7])               # training targets
    te_d = np.concatenate([tr_d, [8, 3]])    # prediction drugs: training ones, then new
    te_t = np.concatenate([tr_t, [0, 6, 1]])
    D = Xd[te_d] @ Xd[tr_d].T                # 6 x 4 linear drug kernel
    T = Xt[te_t] @ Xt[tr_t].T                # 6 x 3 linear target kernel
    n, n_out = 15, 12
    c = r.integers(0, len(tr_d), n).astype(np.int32); e = r.integers(0, len(tr_t), n).astype(np.int32)
    a = r.integers(0, len(te_d), n_out).astype(np.int32); b = r.integers(0, len(te_t), n_out).astype(np.int32)
    a[:3] = [0, 5, 2]; b[:3] = [4, 1, 0]     # shared and new objects on both sides
    v = r.standard_normal(n)
    Kf = _cartesian_feature_kernel(Xd, Xt, te_d[a], te_t[b], tr_d[c], tr_t[e])
    np.testing.assert_allclose(oracle.kernel_matrix("cartesian", D, T, (a, b), (c, e)), Kf,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.pairwise_matvec("cartesian", D, T, (a, b), (c, e), v), Kf @ v,
                               rtol=1e-12, atol=1e-12)
    # new objects only match nothing: their delta terms vanish (R16)
    only_new = (te_d[a] == 8) | (te_d[a] == 3)
    assert only_new.any()
    # the same objects listed in another order on the prediction side break the index reading
    perm = np.array([1, 0, 2, 3, 4, 5])
    D2 = Xd[te_d[perm]] @ Xd[tr_d].T
    Kf2 = _cartesian_feature_kernel(Xd, Xt, te_d[perm][a], te_t[b], tr_d[c], tr_t[e])
    assert not np.allclose(oracle.kernel_matrix("cartesian", D2, T, (a, b), (c, e)), Kf2)
