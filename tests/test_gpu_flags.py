"""The tr_params flags and the device status word, end to end on the GPU.

* TR_FLAG_STABILIZED_POWER: the R-accumulated power scheme against the
  oracle's own stabilised form (oracle.power_sketch_stabilised: Householder QR
  after every step, Rbar = R_q ... R_0, SVD of Rbar) and against the literal
  products: the three are equal in exact arithmetic.  Float64 bar 1e-10 on
  well-separated spectra (factors with canonical signs, core, singular values);
  at full size the kappa-scaled bar of the full-size tests.
* TR_FLAG_UNFUSED_POWER: the two-product form of every power step against the
  one-sweep kernel on shapes where that kernel runs (I <= 128, s <= 32): the
  same sums in another order, 1e-12 relative.
* A NaN planted in the input reaches the status word (TR_DEV_NONFINITE) for
  exact and nearly-optimal sampled products; the call still completes.
* A mode with more than 128 rows and at most 128 columns takes the two-product
  power step with a single column range, whose product kernel writes the
  sketch (and the status) itself: parity with the oracle at 1e-10 for q = 1,
  2 in both power-scheme forms, and a NaN still reaches the status word.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2303_11612_amd as tr
from paper_2303_11612_amd import _abi

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _gpu(A, algo, ranks, K, q, prob="none", samples=None, seed=0, flags=0, precision="native"):
    f = tr.tucker_rand_thosvd if algo == "thosvd" else tr.tucker_rand_sthosvd
    Qs, core, info = f(tr.to_device(A), ranks, K, q, prob, samples, seed, precision=precision,
                       diag=True, flags=flags)
    torch.cuda.synchronize()
    return [_np(Q) for Q in Qs], _np(core), info


STAB_CASES = [
    # shape, true ranks, ranks, K, q, prob, samples
    ((40, 36, 30), (5, 5, 5), (4, 4, 4), 4, 1, "none", None),
    ((40, 36, 30), (5, 5, 5), (4, 4, 4), 4, 3, "none", None),
    ((150, 40, 37), (6, 6, 6), (6, 5, 5), 6, 2, "none", None),
    ((60, 50, 40), (6, 6, 6), (5, 5, 5), 5, 2, "nearly_optimal", (900, 500, 300)),
    ((18, 14, 12, 10), (4, 4, 3, 3), (3, 3, 2, 2), 3, 2, "uniform", (60, 50, 40, 30)),
    # s = 56 > 48: the LDS-resident factor kernel for every orthonormalisation
    # and for Rbar (no transposed copy asked of it there)
    ((80, 70, 60), (40, 40, 40), (40, 40, 40), 16, 2, "none", None),
]


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("case", range(len(STAB_CASES)))
def test_stabilized_power_matches_oracle(algo, case):
    shape, true_r, ranks, K, q, prob, samples = STAB_CASES[case]
    # a graded core with a clear gap after the kept rank, so that the factors
    # are well determined (each column to ~1e-12)
    A = synth.low_rank_plus_noise(shape, true_r, 1e-2, 30 + case)
    Qg, cg, info = _gpu(A, algo, ranks, K, q, prob, samples, 4, flags=["stabilized_power"])
    assert int(_np(info["status"])[0]) == 0
    fo = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qs, cs, infs = fo(A, ranks, K, q, prob, samples, 4, stabilised=True)
    Ql, cl, infl = fo(A, ranks, K, q, prob, samples, 4)
    for n in range(A.ndim):
        assert _rel(Qg[n], Qs[n]) <= 1e-10, (n, _rel(Qg[n], Qs[n]))
        assert _rel(Qg[n], Ql[n]) <= 1e-10, n
        sig = infs[n]["sigma"]
        assert np.allclose(_np(info["sigma"][n]), sig, rtol=1e-9, atol=1e-12 * sig[0]), n
        # the sketch reported is Z_q Rbar, the literal C_n in exact arithmetic
        C = _np(info["sketch"][n])
        assert _rel(C, infl[n]["C"]) <= 1e-9, (n, _rel(C, infl[n]["C"]))
    assert _rel(cg, cs) <= 1e-10
    assert _rel(cg, cl) <= 1e-10


@pytest.mark.parametrize("variant", ["reg", "lds"])
@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_stabilized_power_both_factor_kernels(algo, variant, monkeypatch):
    """The register-resident factor kernel orthonormalises each iterate by its
    Householder QR (and the accumulated triangular factor then skips its own
    QR); the LDS-resident one, forced here for every shape, returns the SVD
    basis and factors a full Rbar.  Either way C_n, the factors and the core
    match the oracle's stabilised form."""
    monkeypatch.setenv("TUCKER_RAND_FACTOR", variant)
    shape, true_r, ranks, K, q, prob, samples = STAB_CASES[2]
    A = synth.low_rank_plus_noise(shape, true_r, 1e-2, 32)
    Qg, cg, info = _gpu(A, algo, ranks, K, q, prob, samples, 4, flags=["stabilized_power"])
    assert int(_np(info["status"])[0]) == 0
    fo = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qs, cs, infs = fo(A, ranks, K, q, prob, samples, 4, stabilised=True)
    for n in range(A.ndim):
        assert _rel(Qg[n], Qs[n]) <= 1e-10, (n, _rel(Qg[n], Qs[n]))
        sig = infs[n]["sigma"]
        assert np.allclose(_np(info["sigma"][n]), sig, rtol=1e-9, atol=1e-12 * sig[0]), n
        assert _rel(_np(info["sketch"][n]), infs[n]["C"]) <= 1e-9, n
    assert _rel(cg, cs) <= 1e-10


def test_stabilized_power_full_size_400cube_q2():
    """400^3 float32, Alg. 1 exact, q = 2, stabilised: against both oracle forms
    with the kappa-scaled bar (projector distance <= max(1e-4, 1e2 u64 kappa_n))."""
    w = synth.config(2)
    Qg, cg, info = _gpu(w.A, "thosvd", (10, 10, 10), 10, 2, flags=["stabilized_power"])
    Qs, cs, infs = oracle.rand_thosvd(w.A, (10, 10, 10), 10, 2, stabilised=True)
    Ql, cl, infl = oracle.rand_thosvd(w.A, (10, 10, 10), 10, 2)
    for n in range(3):
        sig = infl[n]["sigma"]
        kappa = sig[0] / (sig[9] - sig[10])
        bar = max(1e-4, 1e2 * 2.0 ** -53 * kappa)
        Qn = Qg[n].astype(np.float64)
        for Qo in (Qs[n], Ql[n]):
            d = np.linalg.norm(Qn - Qo @ (Qo.T @ Qn), 2)
            assert d <= bar, (n, d, bar)
    re_g = oracle.relative_error(w.A, cg.astype(np.float64), [Q.astype(np.float64) for Q in Qg])
    re_o = oracle.relative_error(w.A, cl, Ql)
    assert abs(re_g - re_o) <= 1e-7, (re_g, re_o)


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
@pytest.mark.parametrize("q", [1, 2])
def test_unfused_power_equals_fused(algo, q):
    # I_n <= 128 and s_n <= 32: the one-sweep kernel applies to every exact mode
    A = synth.low_rank_plus_noise((100, 90, 70), (8, 8, 8), 1e-3, 12)
    Qf, cf, inf_f = _gpu(A, algo, (6, 6, 6), 10, q)
    Qu, cu, inf_u = _gpu(A, algo, (6, 6, 6), 10, q, flags=["unfused_power"])
    for n in range(3):
        assert _rel(_np(inf_u["sketch"][n]), _np(inf_f["sketch"][n])) <= 1e-12, n
        assert _rel(Qu[n], Qf[n]) <= 1e-10, n
    assert _rel(cu, cf) <= 1e-10


def test_unknown_flag_bits_rejected():
    A = tr.to_device(synth.low_rank_plus_noise((20, 10, 5), (2, 2, 2), 0.1, 0))
    with pytest.raises(_abi.TuckerRandError, match="invalid argument"):
        tr.tucker_rand_thosvd(A, (2, 2, 2), 2, 1, flags=0x8)


@pytest.mark.parametrize("prob", ["none", "nearly_optimal"])
@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_nan_input_sets_status(prob, algo):
    A = synth.low_rank_plus_noise((30, 24, 20), (4, 4, 4), 1e-2, 7)
    A[3, 5, 7] = np.nan
    samples = None if prob == "none" else (200, 150, 100)
    _, _, info = _gpu(A, algo, (3, 3, 3), 3, 1, prob, samples, 1)
    assert int(_np(info["status"])[0]) & _abi.TR_DEV_NONFINITE


def test_finite_input_leaves_status_clear():
    A = synth.low_rank_plus_noise((30, 24, 20), (4, 4, 4), 1e-2, 7)
    for prob, samples in (("none", None), ("nearly_optimal", (200, 150, 100))):
        _, _, info = _gpu(A, "sthosvd", (3, 3, 3), 3, 1, prob, samples, 1)
        assert int(_np(info["status"])[0]) == 0


# mode 1 has I = 300 > 128 rows (no one-sweep kernel) and J = 10 * 12 = 120
# columns (one column range): the step's product writes the sketch itself
SINGLE_RANGE_SHAPE = (300, 10, 12)


@pytest.mark.parametrize("flags", [0, ["stabilized_power"]])
@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_single_range_power_step_matches_oracle(algo, q, flags):
    A = synth.low_rank_plus_noise(SINGLE_RANGE_SHAPE, (5, 4, 4), 1e-2, 21)
    ranks, K = (4, 3, 3), 4
    Qg, cg, info = _gpu(A, algo, ranks, K, q, seed=6, flags=flags)
    assert int(_np(info["status"])[0]) == 0
    fo = oracle.rand_thosvd if algo == "thosvd" else oracle.rand_sthosvd
    Qo, co, infos = fo(A, ranks, K, q, "none", None, 6)
    for n in range(A.ndim):
        assert _rel(Qg[n], Qo[n]) <= 1e-10, (n, _rel(Qg[n], Qo[n]))
        assert _rel(_np(info["sketch"][n]), infos[n]["C"]) <= 1e-9, n
    assert _rel(cg, co) <= 1e-10


@pytest.mark.parametrize("algo", ["thosvd", "sthosvd"])
def test_single_range_power_step_nan_sets_status(algo):
    A = synth.low_rank_plus_noise(SINGLE_RANGE_SHAPE, (5, 4, 4), 1e-2, 21)
    A[200, 3, 5] = np.nan
    _, _, info = _gpu(A, algo, (4, 3, 3), 4, 1, seed=6)
    assert int(_np(info["status"])[0]) & _abi.TR_DEV_NONFINITE
