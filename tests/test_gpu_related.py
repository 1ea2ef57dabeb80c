"""GPU parity of the related forms (TR_FLAG_RELATED_FORM: Alg. 6 for T-HOSVD,
Alg. 7 for ST-HOSVD, and the same change to the sampled Alg. 4 / Alg. 5)
against the oracle's related forms on the same inputs and seed.

The device takes P_n as the s_n left singular vectors of C_n (the oracle: the
Householder Q of C_n; both span range(C_n), which fixes Q_n in exact
arithmetic) and U_n as the leading eigenvectors of P_n^T A_(n) A_(n)^T P_n
(the oracle: the SVD of P_n^T A_(n)).  The eigenvectors of that Gram matrix
move by about u64 kappa_rel with kappa_rel = s_1^2 / (s_mu^2 - s_{mu+1}^2),
s_k the singular values of P_n^T A_(n) (the oracle's); and range(C_n) itself
is fixed only to about u64 kappa_C in its weakest direction, kappa_C =
sigma_1(C_n) / sigma_s(C_n), which the related form sees through
P_n^T A_(n) (the plain form does not: it keeps only the leading directions
of C_n).  The bar per mode is max(base, 1e2 u64 (kappa_rel + kappa_C)) on the
projector distance (base 1e-10 for float64
outputs, 1e-4 for float32), columns with canonical signs within that bar
times sqrt(mu) when it is below 1e-6, the rotation-free core within the
largest bar, RE within the sum of the per-mode bars (the multilinear projector
moves by at most that much; at least 1e-10 float64 / 1e-7 float32 outputs), and
the singular values of C_n at 1e-9 relative (same sketch as the plain form).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2303_11612_amd as tr

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _np(t):
    return t.detach().cpu().numpy()


def _pdist(Qa, Qb):
    return float(max(np.linalg.norm(Qa - Qb @ (Qb.T @ Qa), 2),
                     np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2)))


def _compare_related(A, algo, ranks, K, q, prob="none", samples=None, seed=0, flags=()):
    f = tr.tucker_rand_thosvd if algo == "thosvd" else tr.tucker_rand_sthosvd
    Qs, core, info = f(tr.to_device(A), ranks, K, q, prob, samples, seed, diag=True,
                       flags=("related_form",) + tuple(flags))
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) == 0
    Qg = [_np(Q).astype(np.float64) for Q in Qs]
    cg = _np(core).astype(np.float64)
    fo = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qo, co, infos = fo(A, ranks, K, q, prob, samples, seed, related=True)
    f32 = A.dtype == np.float32
    base = 1e-4 if f32 else 1e-10
    bars, carried = [], base
    for n in range(A.ndim):
        sr = infos[n]["sigma_related"]
        mu = ranks[n]
        nxt = sr[mu] if mu < len(sr) else 0.0
        kap = sr[0] ** 2 / max(sr[mu - 1] ** 2 - nxt ** 2, 1e-300)
        sc = infos[n]["sigma"]
        kap_c = sc[0] / max(sc[-1], 1e-300 * sc[0])
        bar = max(base, 1e2 * U64 * (kap + kap_c))
        if algo == "sthosvd":
            bar = max(bar, carried)
            carried = bar
        bars.append(bar)
        d = _pdist(Qg[n], Qo[n])
        assert d <= bar, (n, kap, bar, d)
        if bar < 1e-6:
            cerr = np.linalg.norm(Qg[n] - Qo[n]) / np.linalg.norm(Qo[n])
            assert cerr <= bar * np.sqrt(mu), (n, cerr, bar)
        if prob == "none" or infos[n]["exact"]:
            sig = infos[n]["sigma"]
            assert np.all(np.abs(_np(info["sigma"][n]) - sig) <= 1e-9 * sig + 1e-11 * sig[0]), n
    cr = co
    for n in range(A.ndim):
        cr = oracle.mode_product(cr, Qg[n].T @ Qo[n], n)
    cerr = np.linalg.norm(cg - cr) / np.linalg.norm(co)
    assert cerr <= max(bars), (cerr, max(bars))
    re_g = oracle.relative_error(A, cg, Qg)
    re_o = oracle.relative_error(A, co, Qo)
    # RE = ||A - (P_1 o ... o P_N) A|| / ||A|| moves by at most
    # ||P - P'|| <= sum_n ||P_n - P_n'||: the per-mode projector bars add up
    assert abs(re_g - re_o) <= max(1e-7 if f32 else 1e-10, sum(bars)), (re_g, re_o, sum(bars))
    return re_g, re_o


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("prob,samples", [("none", None), ("nearly_optimal", (500, 300, 200)),
                                          ("uniform", (500, 300, 200))])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_related_small(algo, prob, samples, dtype):
    A = synth.low_rank_plus_noise((41, 33, 27), (6, 6, 5), 1e-2, 61, dtype)
    _compare_related(A, algo, (5, 5, 4), 4, 1, prob, samples, seed=3)


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("q", [2, 3])
def test_related_power_and_stabilized(algo, q):
    A = synth.low_rank_plus_noise((150, 40, 37), (6, 6, 6), 1e-2, 62)
    _compare_related(A, algo, (6, 5, 5), 6, q, seed=4)
    _compare_related(A, algo, (6, 5, 5), 6, q, seed=4, flags=("stabilized_power",))


@pytest.mark.parametrize("flags", [(), ("stabilized_power",)])
def test_related_wide_sketch(flags):
    # s = 56 > 48: the Gram's eigenvectors (and with R-accumulation Rbar's
    # factor) come from the LDS-resident factor kernel, with no transposed copy
    A = synth.low_rank_plus_noise((80, 70, 60), (40, 40, 40), 1e-2, 36)
    _compare_related(A, "thosvd", (40, 40, 40), 16, 2, seed=5, flags=flags)


def test_related_fourth_order_and_k_zero():
    A = synth.low_rank_plus_noise((18, 14, 12, 10), (4, 4, 3, 3), 1e-2, 63)
    _compare_related(A, "sthosvd", (3, 3, 2, 2), 3, 2, "nearly_optimal", (60, 50, 40, 9), seed=8)
    _compare_related(A, "thosvd", (3, 3, 2, 2), 0, 1, seed=8)


def test_related_full_size_400cube_alg7():
    """Alg. 7 on the 400^3 float32 benchmark tensor, exact and with the
    benchmark's sampling (the related form of Alg. 5)."""
    w = synth.config(2)
    _compare_related(w.A, "sthosvd", w.ranks, w.oversample, 1)
    _compare_related(w.A, "sthosvd", w.ranks, w.oversample, 1, w.prob, w.samples, w.seed)


def test_related_full_size_400cube_alg6():
    w = synth.config(2)
    _compare_related(w.A, "thosvd", w.ranks, w.oversample, 1)
