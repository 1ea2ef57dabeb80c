"""Pins of the oracle's related forms (Alg. 6 / Alg. 7, and the same change to
Alg. 4 / Alg. 5) against what the mathematics fixes, not against a retyping:

* optimality: Q_n = P_n U_n is the best mu-dimensional subspace inside
  range(P_n) for A_(n) (Eckart-Young applied to P_n^T A_(n)), so no other
  such subspace -- random ones, or the plain Q_n of Alg. 1 from the same
  sketch -- has a smaller residual ||A_(n) - Q Q^T A_(n)||_F;
* the deterministic bound the paper gives for Alg. 6 (from Gu's subspace
  iteration analysis): ||B - Q Q^T B||_F^2 <= ||S2||_F^2 +
  tau^(4q-1) ||S2 Om2 Om1^+||_F^2 with B = A_(n) = U diag(S) V^T, S1/S2 the
  leading mu / trailing singular values, Om1 = U_1^T G_n, Om2 = U_2^T G_n and
  tau = sigma_{mu+1} / sigma_mu;
* K = 0: P_n spans the range of C_n itself, so the related Q_n spans the same
  subspace as the plain one (projectors equal);
* exact multilinear rank recovered exactly; Eq. (23) for Alg. 7;
* more samples than columns: the sampled related form equals the exact one.
"""
import numpy as np
import pytest

import oracle
import synth


def _resid(An, Q):
    return np.linalg.norm(An - Q @ (Q.T @ An))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("q", [1, 2])
def test_related_factor_is_optimal_inside_range_of_P(seed, q):
    A = synth.low_rank_plus_noise((24, 20, 18), (6, 6, 6), 0.3, 50 + seed)
    mu, K = 4, 5
    rng = np.random.default_rng(seed)
    for n in range(3):
        Qr, info = oracle.range_finder(A, n, mu, K, q, "none", None, seed, related=True)
        Qp, _ = oracle.range_finder(A, n, mu, K, q, "none", None, seed)
        An = oracle.unfold(A, n)
        P = info["P"]
        best = _resid(An, Qr)
        # the plain Q_n lies in range(P_n) too
        assert np.linalg.norm(Qp - P @ (P.T @ Qp)) < 1e-10
        assert best <= _resid(An, Qp) * (1 + 1e-12)
        for _ in range(200):
            V, _ = np.linalg.qr(P @ rng.standard_normal((P.shape[1], mu)))
            assert best <= _resid(An, V) * (1 + 1e-12)
        # the singular values reported are those of P^T A_(n)
        assert np.allclose(info["sigma_related"],
                           np.linalg.svd(P.T @ An, compute_uv=False), rtol=1e-12)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("q", [1, 2, 3])
def test_alg6_deterministic_bound(seed, q):
    A = synth.low_rank_plus_noise((30, 22, 16), (7, 7, 7), 0.2, 70 + seed)
    mu, K = 5, 4
    for n in range(3):
        Q, info = oracle.range_finder(A, n, mu, K, q, "none", None, seed, related=True)
        B = oracle.unfold(A, n)
        U, S, _ = np.linalg.svd(B, full_matrices=False)
        G = info["G"]
        Om1 = U[:, :mu].T @ G
        Om2 = U[:, mu:].T @ G
        S2 = S[mu:]
        tau = S[mu] / S[mu - 1]
        lhs = _resid(B, Q) ** 2
        rhs = np.sum(S2 ** 2) + tau ** (4 * q - 1) * np.linalg.norm(
            (S2[:, None] * Om2) @ np.linalg.pinv(Om1)) ** 2
        assert lhs <= rhs * (1 + 1e-10), (n, lhs, rhs)
        # and never below the Eckart-Young optimum
        assert lhs >= np.sum(S2 ** 2) * (1 - 1e-10)


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_related_with_no_oversampling_spans_the_plain_subspace(algo):
    A = synth.low_rank_plus_noise((20, 16, 14), (5, 5, 5), 0.1, 3)
    f = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qp, cp, _ = f(A, (4, 4, 4), 0, 1, seed=2)
    Qr, cr, _ = f(A, (4, 4, 4), 0, 1, seed=2, related=True)
    for a, b in zip(Qp, Qr):
        assert np.linalg.norm(a @ a.T - b @ b.T, 2) < 1e-10
    assert abs(oracle.relative_error(A, cp, Qp) - oracle.relative_error(A, cr, Qr)) < 1e-12


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("prob,samples", [("none", None), ("nearly_optimal", (200, 180, 150))])
def test_related_recovers_exact_multilinear_rank(algo, prob, samples):
    A = synth.low_rank_plus_noise((28, 24, 20), (4, 5, 3), 0.0, 13)
    f = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qs, core, _ = f(A, (4, 5, 3), 3, 1, prob, samples, seed=5, related=True)
    assert oracle.relative_error(A, core, Qs) < 1e-12
    for Q in Qs:
        assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)


def test_alg7_eq23_bound():
    A = synth.low_rank_plus_noise((15, 13, 11, 6), (4, 4, 3, 3), 0.2, 4)
    ranks = (3, 3, 2, 2)
    Qs, core, _ = oracle.rand_sthosvd(A, ranks, 2, 1, seed=5, related=True)
    re2 = oracle.relative_error(A, core, Qs) ** 2
    X = np.asarray(A)
    bound = 0.0
    for n, Q in enumerate(Qs):
        bound += oracle.frobenius(oracle.mode_product(X, np.eye(Q.shape[0]) - Q @ Q.T, n)) ** 2
        X = oracle.mode_product(X, Q.T, n)
    assert re2 <= bound / oracle.frobenius(A) ** 2 * (1 + 1e-12)


def test_sampled_related_with_more_samples_than_columns_is_exact():
    A = synth.low_rank_plus_noise((20, 12, 6), (4, 4, 3), 1e-2, 6)
    Qe, ce, _ = oracle.rand_sthosvd(A, (4, 3, 2), 3, 1, seed=2, related=True)
    Qs, cs, _ = oracle.rand_sthosvd(A, (4, 3, 2), 3, 1, "uniform", (10**4,) * 3, seed=2,
                                    related=True)
    for a, b in zip(Qe, Qs):
        assert np.array_equal(a, b)
    assert np.array_equal(ce, cs)
