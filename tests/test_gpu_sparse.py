"""GPU parity of the sparse-input ST-HOSVD (tucker_rand_sthosvd_csc, Alg. 5
with the first mode read from compressed sparse columns).

* Against the dense library call on the same tensor: the column norms sum
  each column's nonzeros in row order (the zeros the dense kernel adds change
  nothing), so the draws, the gathered columns, the power products and Q_1
  are bitwise those of tucker_rand_sthosvd; the later factors and the core
  follow from a shrink summed in another order, so both paths are held to
  the oracle's bars.
* Against the oracle on the dense tensor: the bars of the batched tests
  (projector distance within max(base, 1e2 u64 kappa_n) carried through the
  modes, base 1e-10 / 1e-4 for float64 / float32 outputs; rotation-free
  core; RE).
* The paper's sparse 600^3 tensor (Section 6.1, 5 % dense factor vectors):
  Q_1 bitwise equal to the dense path, the library's RE against a float64
  reconstruction.
* An all-zero tensor (nnz = 0) flags TR_DEV_ZERO_DIST; a row index outside
  the mode is skipped and flags TR_DEV_BAD_INDEX.
"""
import numpy as np
import pytest
import torch

import synth
import paper_2303_11612_amd as tr
from paper_2303_11612_amd import _abi
from test_gpu_batch import Case, _check_oracle

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _sparse_case(dims, terms, density, seed, dtype):
    X = synth.sparse_cp_device(dims, terms, density, 1000.0, seed, dtype=dtype)
    return X, synth.csc_mode1(X)


def _run_both(X, csc, ranks, K, q, prob, samples, seed):
    Qs, core, info = tr.tucker_rand_sthosvd_csc(*csc, X.shape, ranks, K, q, prob, samples,
                                                seed, diag=True)
    Qd, cd, infod = tr.tucker_rand_sthosvd(X, ranks, K, q, prob, samples, seed, diag="norms")
    torch.cuda.synchronize()
    return Qs, core, info, Qd, cd, infod


@pytest.mark.parametrize("prob", ["nearly_optimal", "uniform"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sparse_equals_dense_first_factor(prob, dtype):
    X, csc = _sparse_case((90, 70, 60), 90, 0.1, 21, dtype)
    ranks, samples = (8, 7, 6), (1500, 300, 60)
    Qs, core, info, Qd, cd, infod = _run_both(X, csc, ranks, 6, 1, prob, samples, 3)
    assert int(_np(info["status"])[0]) == 0
    assert torch.equal(Qs[0], Qd[0])
    # the later modes see a shrunk tensor summed in another order: both paths
    # are held to the oracle's kappa-scaled bars
    case = Case(_np(X), ranks, samples, 6, 1, prob, 3)
    _check_oracle(case, [_np(Q) for Q in Qs], _np(core))
    _check_oracle(case, [_np(Q) for Q in Qd], _np(cd))
    # ||A||^2 from the same column norms (nearly-optimal) or from the stored
    # values' squares (uniform; the dense path sums every entry)
    a2s, a2d = float(_np(info["norms"])[0]), float(_np(infod["norms"])[0])
    assert abs(a2s - a2d) <= 1e-12 * a2d


@pytest.mark.parametrize("prob", ["nearly_optimal", "uniform"])
def test_sparse_against_oracle(prob):
    X, csc = _sparse_case((80, 64, 50), 80, 0.15, 22, torch.float64)
    A = _np(X)
    ranks, samples, K, seed = (6, 6, 5), (1200, 250, 40), 5, 4
    Qs, core, info = tr.tucker_rand_sthosvd_csc(*csc, X.shape, ranks, K, 1, prob, samples, seed,
                                                diag=True)
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) == 0
    _check_oracle(Case(A, ranks, samples, K, 1, prob, seed), [_np(Q) for Q in Qs], _np(core))


def test_sparse_order4():
    X, csc = _sparse_case((30, 24, 20, 16), 30, 0.2, 23, torch.float64)
    A = _np(X)
    ranks, samples = (5, 5, 4, 4), (800, 300, 120, 60)
    Qs, core, info = tr.tucker_rand_sthosvd_csc(*csc, X.shape, ranks, 4, 2, "nearly_optimal",
                                                samples, 6, diag=True)
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) == 0
    _check_oracle(Case(A, ranks, samples, 4, 2, "nearly_optimal", 6), [_np(Q) for Q in Qs],
                  _np(core))


def test_sparse_paper_600cube():
    """Section 6.1's sparse tensor: 600 rank-one terms of 5 %-dense factor
    vectors (gamma 1000), mu 30, K 10, q 1, alpha 0.01 (uniform, as the
    paper's Alg. 5)."""
    X, csc = _sparse_case((600, 600, 600), 600, 0.05, 24, torch.float32)
    ranks = (30, 30, 30)
    samples = synth.eq9_samples(0.01, X.shape, ranks, True)
    Qs, core, info, Qd, cd, infod = _run_both(X, csc, ranks, 10, 1, "uniform", samples, 5)
    assert int(_np(info["status"])[0]) == 0
    assert torch.equal(Qs[0], Qd[0])
    B = core.double()
    for n, Q in enumerate(Qs):
        B = torch.movedim(torch.tensordot(Q.double(), B, dims=([1], [n])), 0, n)
    A = X.double()
    re = float(torch.linalg.vector_norm(A - B) / torch.linalg.vector_norm(A))
    assert abs(float(_np(info["norms"])[2]) - re) <= 3e-7, (re, float(_np(info["norms"])[2]))


def test_sparse_zero_tensor_and_bad_index():
    dims = (20, 10, 5)
    colptr = torch.zeros(51, dtype=torch.int64, device="cuda")
    rowidx = torch.zeros(0, dtype=torch.int32, device="cuda")
    vals = torch.zeros(0, dtype=torch.float64, device="cuda")
    _, _, info = tr.tucker_rand_sthosvd_csc(colptr, rowidx, vals, dims, (2, 2, 2), 2, 1,
                                            "nearly_optimal", (10, 10, 10), 0, diag=True)
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) & _abi.TR_DEV_ZERO_DIST
    # one nonzero per column, the last column's row index one past the mode
    colptr = torch.arange(51, dtype=torch.int64, device="cuda")
    rowidx = torch.arange(50, dtype=torch.int32, device="cuda") % 20
    rowidx[49] = 20
    vals = torch.ones(50, dtype=torch.float64, device="cuda")
    _, _, info = tr.tucker_rand_sthosvd_csc(colptr, rowidx, vals, dims, (2, 2, 2), 2, 1,
                                            "uniform", (50, 10, 10), 0, diag=True)
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) & _abi.TR_DEV_BAD_INDEX
