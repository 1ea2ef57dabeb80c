"""Pins of the oracle's fixed-precision rule (Problem 2) against what fixes it
independently:

* full-width sketch (s_n = I_n): range(P_n) is the whole space, so the
  squared singular values of P_n^T X_(n) are those of X_(n) and the rule
  reduces to the textbook truncation of the (sequentially) truncated HOSVD
  with an error budget -- recomputed here from full SVDs of the unfoldings;
* exact multilinear rank and a tiny tolerance: the true ranks come back and
  the error is within it; a tolerance of sqrt(N) ||A|| gives rank 1 everywhere;
* the certified bound (Eq. (5) / Eq. (23)) is never below the true error, and
  the true error is within the tolerance whenever the bound is;
* a smaller tolerance never gives a smaller T-HOSVD rank.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _svd_ranks(A, eps, max_ranks, sthosvd):
    """Truncated (ST-)HOSVD ranks from full SVDs: per mode the smallest mu
    whose tail sum of squared singular values fits the same budget."""
    X = np.asarray(A, dtype=np.float64)
    N = X.ndim
    used, mus = 0.0, []
    for n in range(N):
        An = oracle.unfold(X, n)
        U, s, _ = np.linalg.svd(An, full_matrices=False)
        budget = (eps ** 2 - used) / (N - n) if sthosvd else eps ** 2 / N
        mu = max_ranks[n]
        for m in range(1, max_ranks[n] + 1):
            if np.sum(s[m:] ** 2) <= budget:
                mu = m
                break
        used += float(np.sum(s[mu:] ** 2))
        mus.append(mu)
        if sthosvd:
            X = oracle.mode_product(X, U[:, :mu].T, n)
    return mus


@pytest.mark.parametrize("sthosvd", [False, True])
@pytest.mark.parametrize("rel", [0.3, 0.1, 0.03, 0.01])
def test_full_width_sketch_reduces_to_truncated_hosvd(sthosvd, rel):
    A = synth.low_rank_plus_noise((12, 10, 9), (5, 4, 4), 0.05, 7)
    eps = rel * oracle.frobenius(A)
    Qs, core, mus, bound = oracle.rand_tucker_adaptive(A, eps, (12, 10, 9), 20, 1,
                                                       seed=3, sthosvd=sthosvd)
    assert mus == _svd_ranks(A, eps, (12, 10, 9), sthosvd)
    err = oracle.frobenius(A - oracle.reconstruct(core, Qs))
    assert err <= bound * (1 + 1e-10) + 1e-12 and bound <= eps * (1 + 1e-10)


@pytest.mark.parametrize("sthosvd", [False, True])
@pytest.mark.parametrize("prob,samples", [("none", None), ("nearly_optimal", (300, 200, 150))])
def test_exact_rank_recovered(sthosvd, prob, samples):
    A = synth.low_rank_plus_noise((30, 26, 22), (4, 5, 3), 0.0, 13)
    # the residual ||X||^2 - sum lambda_k is a float64 difference with an
    # absolute error of ~u ||A||^2, so tolerances below ~sqrt(u) ||A|| (1e-8)
    # cannot be certified; 1e-6 is well above that floor
    eps = 1e-6 * oracle.frobenius(A)
    Qs, core, mus, bound = oracle.rand_tucker_adaptive(A, eps, (8, 8, 8), 4, 1, prob, samples,
                                                       seed=5, sthosvd=sthosvd)
    assert mus == [4, 5, 3]
    assert oracle.frobenius(A - oracle.reconstruct(core, Qs)) <= eps
    # eps = sqrt(N) ||A||: every mode's budget is at least ||A||^2
    _, _, mus1, _ = oracle.rand_tucker_adaptive(A, math.sqrt(3) * oracle.frobenius(A),
                                                (8, 8, 8), 4, 1, seed=5, sthosvd=sthosvd)
    assert mus1 == [1, 1, 1]


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("sthosvd", [False, True])
def test_certified_bound_holds(seed, sthosvd):
    A = synth.low_rank_plus_noise((25, 21, 18, 7), (6, 5, 5, 4), 0.1, 20 + seed)
    nA = oracle.frobenius(A)
    for rel in (0.5, 0.2, 0.1, 0.05):
        Qs, core, mus, bound = oracle.rand_tucker_adaptive(A, rel * nA, (10, 10, 10, 6), 5, 1,
                                                           seed=seed, sthosvd=sthosvd)
        err = oracle.frobenius(A - oracle.reconstruct(core, Qs))
        assert err <= bound * (1 + 1e-10) + 1e-12
        if bound <= rel * nA:
            assert err <= rel * nA * (1 + 1e-10)
        for Q in Qs:
            assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)


def test_smaller_tolerance_never_lowers_thosvd_ranks():
    A = synth.low_rank_plus_noise((30, 24, 20), (8, 7, 6), 0.05, 3)
    nA = oracle.frobenius(A)
    prev = [0, 0, 0]
    for rel in (0.5, 0.3, 0.2, 0.1, 0.07, 0.05):
        _, _, mus, _ = oracle.rand_tucker_adaptive(A, rel * nA, (12, 12, 12), 6, 2, seed=1,
                                                   sthosvd=False)
        assert all(m >= p for m, p in zip(mus, prev)), (rel, mus, prev)
        prev = mus
