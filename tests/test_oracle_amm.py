"""Pins for the sampled product of Alg. 3 as used in Alg. 4 / Alg. 5.

* Unbiasedness: E[C' C'^T] = A_(n) A_(n)^T because E[S S^T] = I for
  S ~ RANDSAMPLE (Section 3.2).  Checked entrywise by Monte Carlo with the
  exact per-entry variance of the estimator.
* Expected squared error: E||A A^T - C' C'^T||_F^2
  = (1/T)(sum_j ||a_j||^4 / p_j - ||A A^T||_F^2); for p_j proportional to
  ||a_j||^2 the sum is ||A||_F^4 (the optimal choice for A A^T, Remark after
  Alg. 3).
* Lemma 5 (nearly optimal, beta = 1) and Lemma 6 (uniform) tail bounds.
"""
import math

import numpy as np

import oracle

RNG = np.random.default_rng(77)


def _sampled(An, T, prob, seed, mode=0):
    J = An.shape[1]
    norms = oracle.column_sq_norms(An) if prob == oracle.PROB_NEARLY_OPTIMAL else None
    xi, scale, w, W = oracle.randsample(norms, J, T, prob, seed, mode)
    return An[:, xi] * scale[None, :], w, W


def _tensor():
    X = RNG.standard_normal((5, 4, 6)) * np.linspace(0.2, 3.0, 6)[None, None, :]
    return np.asfortranarray(X)


def test_unbiased_entrywise():
    An = oracle.unfold(_tensor(), 0)              # 5 x 24
    exact = An @ An.T
    for prob in (oracle.PROB_NEARLY_OPTIMAL, oracle.PROB_UNIFORM):
        T, M = 16, 1500
        acc = np.zeros_like(exact)
        for seed in range(M):
            Cp, w, W = _sampled(An, T, prob, seed)
            acc += Cp @ Cp.T
        mean = acc / M
        p = w.astype(np.float64) / W
        var = (np.einsum("ij,kj,j->ik", An ** 2, An ** 2, 1.0 / p) - exact ** 2) / T
        z = (mean - exact) / np.sqrt(var / M)
        assert np.max(np.abs(z)) < 5.0, prob


def test_expected_squared_error_and_optimality():
    An = oracle.unfold(_tensor(), 1)              # 4 x 30
    AAt = An @ An.T
    cn = np.sum(An ** 2, axis=0)
    T, M = 12, 1500
    for prob in (oracle.PROB_NEARLY_OPTIMAL, oracle.PROB_UNIFORM):
        errs = []
        for seed in range(M):
            Cp, w, W = _sampled(An, T, prob, seed, mode=1)
            errs.append(np.linalg.norm(AAt - Cp @ Cp.T) ** 2)
        p = w.astype(np.float64) / W
        expect = (np.sum(cn ** 2 / p) - np.linalg.norm(AAt) ** 2) / T
        se = np.std(errs) / math.sqrt(M)
        assert abs(np.mean(errs) - expect) < 4 * se, prob
        if prob == oracle.PROB_NEARLY_OPTIMAL:
            # p ~ ||a_j||^2: sum_j ||a_j||^4 / p_j = ||A||_F^4
            assert math.isclose(np.sum(cn ** 2 / p), np.sum(cn) ** 2, rel_tol=1e-9)


def test_lemma5_and_lemma6_tail_bounds():
    An = oracle.unfold(_tensor(), 2)              # 6 x 20
    AAt = An @ An.T
    delta, T, M = 0.1, 10, 400
    eta = 1 + math.sqrt((8 / delta) * math.log(1 / delta))
    fro2 = np.sum(An ** 2)
    b5 = eta / math.sqrt(T) * fro2                # Lemma 5, beta = 1
    J = An.shape[1]
    cn = np.sqrt(np.sum(An ** 2, axis=0))         # ||A(:,i)|| = ||B(i,:)|| here
    gam = 1 + J / math.sqrt(T) * math.sqrt(8 * math.log(1 / delta)) * np.max(cn ** 2)
    b6 = math.sqrt(J / T) * math.sqrt(np.sum(cn ** 4)) + gam   # Lemma 6
    for prob, bound in ((oracle.PROB_NEARLY_OPTIMAL, b5), (oracle.PROB_UNIFORM, b6)):
        ok = 0
        for seed in range(M):
            Cp, _, _ = _sampled(An, T, prob, seed, mode=2)
            ok += np.linalg.norm(AAt - Cp @ Cp.T) <= bound
        assert ok >= (1 - delta) * M, prob
