"""Pins for the oracle's base kernels from features (Section 5), no GPU.

Linear and Gaussian kernels are checked against library routines (a BLAS product,
scipy's squared Euclidean distances) and closed forms; the Tanimoto kernel against
hand-counted bit vectors and scipy's Jaccard distance on boolean vectors."""
import numpy as np
import pytest

import oracle

scipy_dist = pytest.importorskip("scipy.spatial.distance")


def _pack(bits):
    """Rows of 0/1 values -> rows of uint64 words, bit b in word b // 64 at b % 64."""
    bits = np.asarray(bits, dtype=np.uint8)
    n, nb = bits.shape
    words = (nb + 63) // 64
    out = np.zeros((n, words), dtype=np.uint64)
    for b in range(nb):
        out[:, b // 64] |= bits[:, b].astype(np.uint64) << np.uint64(b % 64)
    return out


def test_linear_is_library_product():
    r = np.random.default_rng(41)
    X, Y = r.standard_normal((13, 7)), r.standard_normal((9, 7))
    np.testing.assert_allclose(oracle.base_kernel("linear", X, Y), X @ Y.T, rtol=1e-13, atol=1e-13)
    K = oracle.base_kernel("linear", X)
    np.testing.assert_allclose(K, X @ X.T, rtol=1e-13, atol=1e-13)
    assert np.array_equal(K, K.T)


def test_gaussian_closed_forms_and_library_distances():
    X = np.array([[0.0, 0.0], [3.0, 4.0], [1.0, -1.0]])
    g = 0.01
    K = oracle.base_kernel("gaussian", X, gamma=g)
    # hand-computed squared distances: 25, 2, 29
    want = np.exp(-g * np.array([[0, 25, 2], [25, 0, 29], [2, 29, 0]], dtype=float))
    np.testing.assert_allclose(K, want, rtol=1e-15)
    assert np.all(np.diag(K) == 1.0)
    r = np.random.default_rng(42)
    X, Y = r.standard_normal((11, 5)), r.standard_normal((8, 5))
    ref = np.exp(-0.3 * scipy_dist.cdist(X, Y, "sqeuclidean"))
    np.testing.assert_allclose(oracle.base_kernel("gaussian", X, Y, gamma=0.3), ref, rtol=1e-13)
    # translation invariance and positive semi-definiteness
    c = r.standard_normal(5)
    np.testing.assert_allclose(oracle.base_kernel("gaussian", X + c, Y + c, gamma=0.3),
                               oracle.base_kernel("gaussian", X, Y, gamma=0.3), rtol=1e-12)
    assert np.linalg.eigvalsh(oracle.base_kernel("gaussian", X, gamma=0.3)).min() > -1e-12


def test_tanimoto_hand_counted():
    #        bits:  0 1 2 3 4 5
    v = np.array([[1, 1, 0, 0, 1, 0],    # {0, 1, 4}
                  [1, 0, 1, 0, 1, 1],    # {0, 2, 4, 5}
                  [0, 0, 0, 0, 0, 0],    # {}
                  [0, 1, 0, 1, 0, 0]])   # {1, 3}
    K = oracle.tanimoto(_pack(v), nbits=6)
    # |A and B| / |A or B| counted by hand
    want = np.array([[1, 2 / 5, 0, 1 / 4],
                     [2 / 5, 1, 0, 0],
                     [0, 0, 1, 0],        # two empty vectors: 1 (reading of 0/0)
                     [1 / 4, 0, 0, 1]])
    assert np.array_equal(K, want)


def test_tanimoto_known_counts_across_words_and_scipy():
    r = np.random.default_rng(43)
    nb = 150  # three words, a ragged last one
    for inter, only_a, only_b in [(10, 5, 7), (0, 3, 4), (40, 0, 0), (1, 60, 70)]:
        pos = r.permutation(nb)
        a = np.zeros(nb, np.uint8); b = np.zeros(nb, np.uint8)
        a[pos[:inter]] = b[pos[:inter]] = 1
        a[pos[inter:inter + only_a]] = 1
        b[pos[inter + only_a:inter + only_a + only_b]] = 1
        K = oracle.tanimoto(_pack(a[None]), _pack(b[None]), nbits=nb)
        assert K[0, 0] == inter / (inter + only_a + only_b)
    bits = (r.random((12, nb)) < 0.3).astype(np.uint8)
    K = oracle.tanimoto(_pack(bits), nbits=nb)
    ref = 1.0 - scipy_dist.cdist(bits.astype(bool), bits.astype(bool), "jaccard")
    np.testing.assert_allclose(K, ref, rtol=1e-15, atol=1e-15)
    assert np.linalg.eigvalsh(K).min() > -1e-12  # the Tanimoto kernel is PSD on binary vectors


def test_tanimoto_ignores_bits_past_nbits():
    a = np.array([[0b1011, 0xFF00]], dtype=np.uint64)   # nbits = 70: only 6 bits of word 1 count
    b = np.array([[0b0011, 0x00FF]], dtype=np.uint64)
    # word 0: a={0,1,3}, b={0,1}; word 1 bits 0..5: a none, b={0..5}
    K = oracle.tanimoto(a, b, nbits=70)
    assert K[0, 0] == 2 / (3 + 6)
