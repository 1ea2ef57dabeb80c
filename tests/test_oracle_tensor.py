"""Pins for the oracle's multilinear algebra (Section 2): unfolding, folding,
mode-n product, column norms.

Fixed by brute-force index loops written from the paper's definitions on small
integer-valued tensors (exact equality), by numpy.einsum, and by the algebraic
rules the paper states for mode products.
"""
import itertools

import numpy as np
import pytest

import oracle


def _int_tensor(shape, seed):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.integers(-9, 10, size=shape).astype(np.float64))


@pytest.mark.parametrize("shape", [(3, 4), (2, 3, 4), (3, 1, 2, 4), (2, 2, 3, 2, 2), (5,)])
def test_unfold_matches_paper_index_map(shape):
    X = _int_tensor(shape, 1)
    N = len(shape)
    for n in range(N):
        An = oracle.unfold(X, n)
        J = int(np.prod([shape[m] for m in range(N) if m != n]))
        assert An.shape == (shape[n], J)
        for idx in itertools.product(*[range(s) for s in shape]):
            # 1-based map of Section 2, j = i_1 + (i_2 - 1) I_1 + ..., skipping mode n
            j1, stride = 1, 1
            for k in range(N):
                if k == n:
                    continue
                j1 += (idx[k] + 1 - 1) * stride
                stride *= shape[k]
            assert An[idx[n], j1 - 1] == X[idx]
        assert np.array_equal(oracle.fold(An, n, shape), X)


def test_mode_product_brute_force():
    X = _int_tensor((3, 4, 2), 2)
    rng = np.random.default_rng(3)
    for n in range(3):
        B = rng.integers(-5, 6, size=(5, X.shape[n])).astype(np.float64)
        Y = oracle.mode_product(X, B, n)
        shp = list(X.shape)
        shp[n] = 5
        assert Y.shape == tuple(shp)
        for idx in itertools.product(*[range(s) for s in shp]):
            acc = 0.0
            for i in range(X.shape[n]):
                src = list(idx)
                src[n] = i
                acc += X[tuple(src)] * B[idx[n], i]
            assert Y[idx] == acc


def test_mode_product_matches_einsum_and_rules():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 5, 6, 3))
    F = rng.standard_normal((2, 5))
    Gm = rng.standard_normal((7, 6))
    H = rng.standard_normal((3, 2))
    e = np.einsum("abcd,jb->ajcd", X, F)
    assert np.allclose(oracle.mode_product(X, F, 1), e, rtol=1e-13, atol=1e-13)
    # commutation for distinct modes and composition on one mode (Section 2)
    a = oracle.mode_product(oracle.mode_product(X, F, 1), Gm, 2)
    b = oracle.mode_product(oracle.mode_product(X, Gm, 2), F, 1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    c = oracle.mode_product(oracle.mode_product(X, F, 1), H, 1)
    d = oracle.mode_product(X, H @ F, 1)
    assert np.allclose(c, d, rtol=1e-12, atol=1e-12)


def test_column_norms_exact_on_integers():
    X = _int_tensor((7, 3, 5), 5)
    for n in range(3):
        An = oracle.unfold(X, n)
        got = oracle.column_sq_norms(An)
        want = [sum(int(v) ** 2 for v in An[:, j]) for j in range(An.shape[1])]
        assert got.tolist() == [float(w) for w in want]


def test_column_norms_accumulate_in_row_order():
    # squares 2^54, 1, 1, 1, 1: adding the ones after 2^54 loses each of them
    # (ulp(2^54) = 4, ties to even), adding them first gives 2^54 + 4.
    col = np.array([[2.0**27], [1.0], [1.0], [1.0], [1.0]])
    assert oracle.column_sq_norms(col)[0] == 2.0**54
    assert oracle.column_sq_norms(col[::-1])[0] == 2.0**54 + 4


def test_frobenius_and_inner_product():
    X = _int_tensor((3, 4, 5), 6)
    assert oracle.frobenius(X) ** 2 == pytest.approx(float(np.sum(X * X)), rel=1e-15)
    for n in range(3):
        assert oracle.column_sq_norms(oracle.unfold(X, n)).sum() == pytest.approx(
            oracle.frobenius(X) ** 2, rel=1e-15)
