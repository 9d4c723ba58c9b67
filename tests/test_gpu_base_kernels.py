"""Base kernel matrices from features on the GPU (Section 5) against the oracle.

Linear and Gaussian: norm-wise relative error 1e-10 (FP64) / 1e-5 (FP32), exact symmetry
and unit diagonal for a sample with itself.  Tanimoto: integer counts, so bit for bit."""
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


def nrel(got, ref):
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / np.linalg.norm(ref))


def _pack(bits):
    bits = np.asarray(bits, dtype=np.uint8)
    n, nb = bits.shape
    out = np.zeros((n, (nb + 63) // 64), dtype=np.uint64)
    for b in range(nb):
        out[:, b // 64] |= bits[:, b].astype(np.uint64) << np.uint64(b % 64)
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["linear", "gaussian"])
@pytest.mark.parametrize("shape", [(1, 1, 3), (300, 200, 37), (129, 257, 64), (70, 70, 0)])
def test_gram_kernels_vs_oracle(gvt, kind, prec, shape):
    nx, ny, dim = shape
    r = np.random.default_rng([51, nx, ny, dim])
    X, Y = r.standard_normal((nx, dim)), r.standard_normal((ny, dim))
    dt = torch.float64 if prec == "f64" else torch.float32
    g = 1.0 / 32
    tol = 1e-10 if prec == "f64" else 1e-5
    K = gvt.gvt_base_kernel(kind, dev(X, dt), dev(Y, dt), gamma=g).double().cpu().numpy()
    ref = oracle.base_kernel(kind, X, Y, gamma=g)
    if np.linalg.norm(ref) == 0:
        assert np.all(K == 0)
    else:
        assert nrel(K, ref) < tol
    # one sample with itself: exactly symmetric; Gaussian diagonal exactly 1
    Ks = gvt.gvt_base_kernel(kind, dev(X, dt), None, gamma=g)
    assert torch.equal(Ks, Ks.t())
    Ks = Ks.double().cpu().numpy()
    refs = oracle.base_kernel(kind, X, gamma=g)
    if np.linalg.norm(refs) > 0:
        assert nrel(Ks, refs) < tol
    if kind == "gaussian":
        assert np.all(np.diag(Ks) == 1.0)


def test_gram_kernel_strided_rows(gvt):
    # row strides above the feature count, in all three matrices
    r = np.random.default_rng(52)
    Xb, Yb = r.standard_normal((150, 40)), r.standard_normal((90, 40))
    X, Y = dev(Xb)[:, :33], dev(Yb)[:, :33]
    out = torch.full((150, 100), -3.0, dtype=torch.float64, device="cuda")
    gvt.gvt_base_kernel("gaussian", X, Y, gamma=0.05, out=out[:, :90])
    ref = oracle.base_kernel("gaussian", Xb[:, :33], Yb[:, :33], gamma=0.05)
    assert nrel(out[:, :90].cpu().numpy(), ref) < 1e-10
    assert torch.all(out[:, 90:] == -3.0)


@pytest.mark.parametrize("nbits", [1, 64, 150, 1024])
@pytest.mark.parametrize("shape", [(5, 7), (130, 70)])
def test_tanimoto_bitwise(gvt, nbits, shape):
    nx, ny = shape
    r = np.random.default_rng([53, nbits, nx])
    bx = (r.random((nx, nbits)) < 0.2).astype(np.uint8)
    by = (r.random((ny, nbits)) < 0.3).astype(np.uint8)
    bx[0] = 0
    by[1] = 0  # empty vectors: Tanimoto 1 against each other, 0 otherwise
    px, py = _pack(bx), _pack(by)
    # garbage above nbits in the last word must be ignored
    if nbits % 64:
        px[:, -1] |= np.uint64(~((1 << (nbits % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
    ref = oracle.tanimoto(px, py, nbits=nbits)
    tx, ty = dev(px.view(np.int64)), dev(py.view(np.int64))
    K = gvt.gvt_tanimoto_kernel(tx, ty, nbits=nbits)
    assert np.array_equal(K.cpu().numpy(), ref)
    K32 = gvt.gvt_tanimoto_kernel(tx, ty, nbits=nbits, dtype=torch.float32)
    assert np.array_equal(K32.cpu().numpy(), ref.astype(np.float32))
    Ks = gvt.gvt_tanimoto_kernel(tx, None, nbits=nbits)
    assert np.array_equal(Ks.cpu().numpy(), oracle.tanimoto(px, nbits=nbits))


def test_base_kernel_argument_errors(gvt):
    import ctypes

    X = dev(np.zeros((4, 3)))
    with pytest.raises(gvt.GvtError) as ei:
        gvt.gvt_base_kernel("gaussian", X, None, gamma=float("nan"))
    assert ei.value.code == -1
    K = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    lib = gvt.load_library()
    assert lib.gvt_base_kernel(7, 0, p(X), 4, 3, None, 4, 0, 3, 0.0, p(K), 4, None) == -1  # unknown kind
    assert lib.gvt_base_kernel(0, 0, p(X), 4, 3, None, 5, 0, 3, 0.0, p(K), 5, None) == -1  # Y = X, ny != nx
    assert lib.gvt_base_kernel(0, 0, p(X), 4, 2, None, 4, 0, 3, 0.0, p(K), 4, None) == -1  # ldx < dim


def test_ridge_features_to_solution(gvt):
    # The ridge workload from its features: D and T built on the GPU (Gaussian, sigma = 4),
    # then the CG solve; against the oracle's base kernels and the host-built solve.
    p = W.config2()
    g = 1.0 / (2.0 * W.SIGMA ** 2)
    D = gvt.gvt_base_kernel("gaussian", dev(p["Xd"]), None, gamma=g)
    T = gvt.gvt_base_kernel("gaussian", dev(p["Xt"]), None, gamma=g)
    rows = np.random.default_rng(54).choice(2000, 64, replace=False)
    refD = oracle.base_kernel("gaussian", p["Xd"][rows], p["Xd"], gamma=g)
    assert nrel(D.cpu().numpy()[rows], refD) < 1e-10
    assert nrel(T.cpu().numpy(), oracle.base_kernel("gaussian", p["Xt"], gamma=g)) < 1e-10
    inp = (dev(p["c"]), dev(p["e"]))
    A, iters, rel, rc = gvt.gvt_krr_cg("kronecker", D, T, inp, dev(p["y"]), [p["lam"]], max_iter=200, tol=1e-6)
    A2, iters2, rel2, rc2 = gvt.gvt_krr_cg("kronecker", dev(p["D"]), dev(p["T"]), inp, dev(p["y"]), [p["lam"]],
                                           max_iter=200, tol=1e-6)
    assert rc == rc2 == 0 and rel[0] < 1e-6
    assert nrel(A[:, 0].cpu().numpy(), A2[:, 0].cpu().numpy()) < 1e-8
