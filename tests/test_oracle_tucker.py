"""Pins for the oracle's drivers (Alg. 1, 2, 4, 5) and range finder.

Each check is fixed by something other than the oracle itself:
* exact recovery of tensors of exact multilinear rank (RE ~ 0, projectors equal
  to those of the full SVD of every unfolding);
* Eckart-Young / Lemma 3 lower bound Delta_{mu+1}(A_(n)) computed by LAPACK SVD;
* convergence of the power scheme to the truncated SVD for large q;
* Q^T Q = I;
* the deterministic error bounds Eq. (5) (T-HOSVD) and Eq. (23) (ST-HOSVD);
* the sqrt(N) bound against the best per-mode truncation;
* the orthogonal-projection identity RE^2 = 1 - ||G||^2 / ||A||^2 (Eq. (8));
* Lemma 8 (singular values of the shrunk unfoldings do not grow);
* Theorem 5's probabilistic bound;
* the N = 2 special case, where the method reduces to the matrix randomized
  range finder, computed here with Strategy B (Remark after Alg. 1);
* T_n > J_n (exact product) equals the unsampled algorithm.
"""
import math

import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(2023)


def _exact_rank_tensor(dims, ranks, seed):
    return synth.low_rank_plus_noise(dims, ranks, 0.0, seed, np.float64)


def _proj(U):
    return U @ U.T


def _left_sv(M, k):
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    return U[:, :k], s


def _tail(s, k):
    """Delta_{k+1} = sqrt(sum_{i > k} sigma_i^2)."""
    return math.sqrt(float(np.sum(s[k:] ** 2)))


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("prob", ["none", "nearly_optimal", "uniform"])
def test_exact_multilinear_rank_recovery(algo, prob):
    dims, ranks = (13, 11, 9), (3, 4, 2)
    A = _exact_rank_tensor(dims, ranks, 7)
    f = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    samples = None if prob == "none" else (60, 60, 60)
    Qs, core, _ = f(A, ranks, 3, 1, prob, samples, seed=11)
    assert oracle.relative_error(A, core, Qs) < 1e-12
    for n in range(3):
        U, _ = _left_sv(oracle.unfold(A, n), ranks[n])
        assert np.linalg.norm(_proj(Qs[n]) - _proj(U), 2) < 1e-10


@pytest.mark.parametrize("seed", range(5))
def test_eckart_young_lower_bound_and_orthonormality(seed):
    A = synth.low_rank_plus_noise((14, 12, 10), (4, 4, 4), 0.05, seed)
    for f in (oracle.rand_thosvd, oracle.rand_sthosvd):
        Qs, core, infos = f(A, (4, 3, 5), 2, 1, seed=seed)
        X = np.asarray(A)
        for n, Q in enumerate(Qs):
            assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-13
            An = oracle.unfold(X, n)
            _, s = _left_sv(An, 1)
            err = np.linalg.norm(An - Q @ (Q.T @ An))
            assert err >= _tail(s, Q.shape[1]) * (1 - 1e-12)
            if f is oracle.rand_sthosvd:
                X = oracle.mode_product(X, Q.T, n)


def test_power_scheme_converges_to_truncated_svd():
    # every unfolding has singular values v; the top-mu left singular vectors
    # of C_n approach those of A_(n) at the rate (sigma_{mu+1}/sigma_mu)^(2q)
    v = [1.0, 0.9, 0.8, 0.7, 0.6, 0.06, 0.05, 0.04, 0.03, 0.02] + [1e-3] * 4
    dims = (30, 28, 26)
    B = synth.low_rank_plus_noise(dims, (14, 14, 14), 0.0, 3, core="tendiag",
                                  decay=v)
    Qs, _, _ = oracle.rand_thosvd(B, (5, 5, 5), 5, 10, seed=3)
    for n in range(3):
        U, s = _left_sv(oracle.unfold(B, n), 5)
        assert np.allclose(s[:14], v, rtol=1e-12)
        assert np.linalg.norm(_proj(Qs[n]) - _proj(U), 2) < 1e-10


def test_strategy_a_equals_strategy_b():
    M = RNG.standard_normal((9, 40))
    G = RNG.standard_normal((9, 4))
    for q in (1, 2, 3):
        a = oracle.power_sketch(M, G, q)
        b = np.linalg.matrix_power(M @ M.T, q) @ G
        assert np.allclose(a, b, rtol=1e-11, atol=1e-11 * np.abs(b).max())


def test_stabilised_equals_literal():
    A = synth.low_rank_plus_noise((20, 18, 16), (5, 5, 5), 0.1, 9)
    for q in (1, 2):
        Q1, _, _ = oracle.rand_sthosvd(A, (4, 4, 4), 4, q, seed=2)
        Q2, _, _ = oracle.rand_sthosvd(A, (4, 4, 4), 4, q, seed=2, stabilised=True)
        for a, b in zip(Q1, Q2):
            assert np.allclose(a, b, atol=1e-11)


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_deterministic_error_bounds_eq5_eq23(algo):
    A = synth.low_rank_plus_noise((15, 13, 11, 6), (4, 4, 3, 3), 0.2, 4)
    ranks = (3, 3, 2, 2)
    f = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qs, core, _ = f(A, ranks, 2, 1, seed=5)
    re2 = oracle.relative_error(A, core, Qs) ** 2
    nA2 = oracle.frobenius(A) ** 2
    X = np.asarray(A)
    bound = 0.0
    for n, Q in enumerate(Qs):
        P = np.eye(Q.shape[0]) - Q @ Q.T
        bound += oracle.frobenius(oracle.mode_product(X, P, n)) ** 2
        if algo == "sthosvd":
            X = oracle.mode_product(X, Q.T, n)   # Eq. (23): current tensor
    assert re2 <= bound / nA2 * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_sqrt_n_times_best_truncation(seed):
    w = synth.config(1, seed)
    A = w.A
    Qs, core, _ = oracle.rand_thosvd(A, w.ranks, w.oversample, w.power, seed=seed)
    re = oracle.relative_error(A, core, Qs)
    deltas = []
    for n in range(3):
        _, s = _left_sv(oracle.unfold(A, n), 1)
        deltas.append(_tail(s, w.ranks[n]))
    nA = oracle.frobenius(A)
    # the best rank-(mu) Tucker error is at least max_n Delta_n / ||A||
    assert re <= math.sqrt(3) * max(deltas) / nA
    # deterministic truncated HOSVD for comparison (large spectral gap here)
    Ud = [_left_sv(oracle.unfold(A, n), w.ranks[n])[0] for n in range(3)]
    cd = A
    for n in range(3):
        cd = oracle.mode_product(cd, Ud[n].T, n)
    assert re <= 1.01 * oracle.relative_error(A, cd, Ud)


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("prob", ["none", "nearly_optimal"])
def test_re_projector_identity(algo, prob):
    A = synth.low_rank_plus_noise((16, 15, 14), (5, 5, 5), 0.05, 8)
    f = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    smp = None if prob == "none" else (40, 40, 40)
    Qs, core, _ = f(A, (4, 4, 4), 3, 1, prob, smp, seed=1)
    re = oracle.relative_error(A, core, Qs)
    ident = 1.0 - oracle.frobenius(core) ** 2 / oracle.frobenius(A) ** 2
    assert abs(re ** 2 - ident) < 1e-12


def test_lemma8_shrunk_singular_values():
    A = synth.low_rank_plus_noise((12, 11, 10, 9), (4, 4, 4, 4), 0.3, 6)
    ranks = (3, 3, 3, 3)
    _, _, infos = oracle.rand_sthosvd(A, ranks, 2, 1, seed=3)
    for n, info in enumerate(infos):
        sB = np.linalg.svd(oracle.unfold(info["X_before"], n), compute_uv=False)
        sA = np.linalg.svd(oracle.unfold(np.asarray(A), n), compute_uv=False)
        k = len(sB)
        assert np.all(sB <= sA[:k] * (1 + 1e-12) + 1e-14)
        assert _tail(sB, ranks[n]) <= _tail(sA, ranks[n]) * (1 + 1e-12)


def test_theorem5_bound_holds():
    # Theorem 5 with gamma = 2, beta = 1 + 1e-9: the failure probability of
    # Eq. (16) is below 1e-2 here; require the bound in >= 90% of seeds.
    dims, mu, K, q = (20, 18, 16), 3, 4, 1
    A = synth.low_rank_plus_noise(dims, (6, 6, 6), 0.3, 12)
    gamma, beta = 2.0, 1.0 + 1e-9
    ok = total = 0
    for seed in range(60):
        Qs, _, _ = oracle.rand_thosvd(A, (mu,) * 3, K, q, seed=seed)
        for n in range(3):
            An = oracle.unfold(np.asarray(A), n)
            I, J = An.shape
            Ip = min(I, J)
            s = np.linalg.svd(An, compute_uv=False)
            dq = math.sqrt(float(np.sum(s[mu:Ip] ** (4 * q))))
            lam = ((math.sqrt(max(Ip - mu, mu + K)) + math.sqrt(I))
                   * math.sqrt(2 * (mu + K)) * gamma * beta / s[mu - 1] ** (2 * q - 1))
            bound = 2 * (lam * dq + _tail(s, mu))
            err = np.linalg.norm(An - Qs[n] @ (Qs[n].T @ An))
            ok += err <= bound
            total += 1
    assert ok >= 0.9 * total


def test_order_two_reduces_to_matrix_range_finder():
    M = RNG.standard_normal((12, 9)) @ np.diag(0.7 ** np.arange(9)) @ \
        RNG.standard_normal((9, 9))
    mu, K, q, seed = 3, 2, 2, 17
    Qs, core, _ = oracle.rand_thosvd(M, (mu, mu), K, q, seed=seed)
    for n, Mat in enumerate((M, M.T)):
        G = oracle.gaussian_matrix(Mat.shape[0], mu + K, n, seed)
        C = np.linalg.matrix_power(Mat @ Mat.T, q) @ G      # Strategy B
        U = np.linalg.svd(C)[0][:, :mu]
        assert np.linalg.norm(_proj(Qs[n]) - _proj(U), 2) < 1e-10
    assert np.allclose(core, Qs[0].T @ M @ Qs[1], atol=1e-12)


def test_sampling_with_more_samples_than_columns_is_exact():
    A = synth.low_rank_plus_noise((10, 9, 3), (3, 3, 2), 0.1, 2)
    Qe, ce, _ = oracle.rand_sthosvd(A, (3, 3, 2), 2, 1, seed=4)
    Qs, cs, infos = oracle.rand_sthosvd(A, (3, 3, 2), 2, 1, "nearly_optimal",
                                        (1000, 1000, 1000), seed=4)
    assert all(i["exact"] for i in infos)
    for a, b in zip(Qe, Qs):
        assert np.array_equal(a, b)
    assert np.array_equal(ce, cs)


def test_canonical_signs():
    Q = oracle.canonical_signs(np.array([[0.1, -0.8], [-0.9, 0.8], [0.2, 0.0]]))
    assert Q[1, 0] == 0.9 and Q[0, 1] == 0.8 and Q[1, 1] == -0.8


def test_sketch_width_is_capped_at_mode_size():
    A = synth.low_rank_plus_noise((6, 30, 30), (3, 3, 3), 0.1, 1)
    _, _, infos = oracle.rand_thosvd(A, (4, 4, 4), 10, 1, seed=0)
    assert [i["s"] for i in infos] == [6, 14, 14]


def test_argument_validation():
    A = np.zeros((5, 4, 3)) + 1.0
    with pytest.raises(ValueError):
        oracle.rand_thosvd(A, (6, 2, 2), 1, 1)
    oracle.rand_sthosvd(A, (2, 2, 3), 1, 1)       # J_3 = 2*2 = 4 >= mu_3 = 3
    with pytest.raises(ValueError):
        oracle.rand_sthosvd(A, (1, 1, 3), 1, 1)   # J_3 = 1*1 < mu_3
    with pytest.raises(ValueError):
        oracle.rand_thosvd(A, (2, 2, 2), 1, 0)
    with pytest.raises(ValueError):
        oracle.rand_thosvd(A, (2, 2, 2), 1, 1, "uniform", (0, 1, 1))
    with pytest.raises(ValueError):
        oracle.rand_thosvd(A, (2, 2, 2), 1, 1, "optimal", (1, 1, 1))
    with pytest.raises(FloatingPointError):
        oracle.rand_thosvd(np.zeros((5, 4, 3)), (2, 2, 2), 1, 1,
                           "nearly_optimal", (3, 3, 3))
