"""The dense product without allocation (static per-device workspace) against the
allocating entry point, through the C ABI, on two calls in a row (the second smaller)."""
import numpy as np
import pytest

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


def _inputs(seed, m, q, dt):
    r = np.random.default_rng([31, seed, m, q])
    D = W.gaussian_kernel(r.standard_normal((m, 8)))
    T = W.gaussian_kernel(r.standard_normal((q, 8)))
    V = r.standard_normal((m, q))
    return [torch.from_numpy(x).to("cuda", dt) for x in (D, T, V)], D @ V @ T.T


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6"])
def test_noalloc_matches_allocating_entry_point(gvt, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    pc = {"f64": gvt.F64, "f32": gvt.F32, "bf16x3": gvt.BF16X3, "bf16x6": gvt.BF16X6}[prec]
    for seed, (m, q) in enumerate([(700, 530), (257, 130)]):  # second call smaller, ragged tiles
        (Dd, Td, Vd), ref = _inputs(seed, m, q, dt)
        want = gvt.gvt_dense_matvec(Dd, Td, Vd, prec=pc)
        got = gvt.gvt_dense_matvec_noalloc(Dd, Td, Vd, prec=pc)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: bitwise equal
        assert torch.equal(got, want), (prec, m, q)
        err = np.linalg.norm(got.cpu().double().numpy() - ref) / np.linalg.norm(ref)
        assert err < {"f64": 1e-10, "f32": 1e-5, "bf16x3": 1e-4, "bf16x6": 1e-5}[prec], (prec, m, q, err)


def test_noalloc_rejects_products_beyond_its_workspace(gvt):
    m, q = 4096, 4096  # W alone is 128 MiB in FP64
    Dd = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    Td = torch.zeros((q, q), dtype=torch.float64, device="cuda")
    Vd = torch.zeros((m, q), dtype=torch.float64, device="cuda")
    with pytest.raises(gvt.GvtError) as ei:
        gvt.gvt_dense_matvec_noalloc(Dd, Td, Vd, prec=gvt.F64)
    assert ei.value.code == -1 and "static workspace" in str(ei.value)
