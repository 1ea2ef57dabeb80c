"""The paper's own synthetic workloads on the GPU.

* The Eq. (9) tensor (core iid U(0,1), orthonormal Gaussian factors, relative
  noise gamma), built on the device by synth.tucker_noise_device, at a reduced
  size the oracle runs in seconds (150^3, core 25^3): Alg. 1, 2, 4 and 5 with
  q 1, K 10, alpha 0.2 and the paper's uniform probabilities, against the
  oracle on the same (copied back) tensor with the bars of
  test_gpu_fullsize (projector distance within max(1e-4, 1e2 u64 kappa_n),
  rotation-free core, RE within 1e-7, the library's RE against the
  reconstruction of its outputs).
* Ranks past 54 (sketch widths 65..128): the Eq. (9) tensor at 200^3 with
  the paper's 100^3 core, mu 80 (s 90), all four algorithms against the
  oracle with the same bars.
* Full size (600^3, mu 50 and mu 100 -- the paper's largest, s = 110): the
  library's RE against a float64 reconstruction of its outputs, orthonormal
  factors, status 0 -- Alg. 2 and Alg. 5.
* The Section 6.3 tendiag tensor at 200^3 (50 unit values then
  (i - 49)^-2): Alg. 2 against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2303_11612_amd as tr
from test_gpu_fullsize import _fullsize_compare

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def eq9_small():
    X = synth.tucker_noise_device((150, 150, 150), (25, 25, 25), 1e-3, 11)
    return _np(X)


@pytest.mark.parametrize("algo,prob", [("thosvd", "none"), ("sthosvd", "none"),
                                       ("thosvd", "uniform"), ("sthosvd", "uniform")])
@pytest.mark.parametrize("mu", [10, 20])
def test_eq9_reduced_against_oracle(eq9_small, algo, prob, mu):
    ranks = (mu,) * 3
    samples = None
    if prob != "none":
        samples = synth.eq9_samples(0.2, eq9_small.shape, ranks, algo == "sthosvd")
    _fullsize_compare(eq9_small, algo, ranks, 10, 1, prob, samples, seed=4)


@pytest.fixture(scope="module")
def eq9_core100():
    return _np(synth.tucker_noise_device((200, 200, 200), (100, 100, 100), 1e-3, 14))


@pytest.mark.parametrize("algo,prob", [("thosvd", "none"), ("sthosvd", "none"),
                                       ("thosvd", "uniform"), ("sthosvd", "uniform")])
def test_eq9_wide_sketch_against_oracle(eq9_core100, algo, prob):
    ranks = (80, 80, 80)
    samples = None
    if prob != "none":
        samples = synth.eq9_samples(0.2, eq9_core100.shape, ranks, algo == "sthosvd")
    _fullsize_compare(eq9_core100, algo, ranks, 10, 1, prob, samples, seed=8)


@pytest.mark.parametrize("mu", [50, 100])
@pytest.mark.parametrize("prob", ["none", "uniform"])
def test_eq9_600cube(prob, mu):
    X = synth.tucker_noise_device((600, 600, 600), (100, 100, 100), 1e-3, 12)
    ranks = (mu, mu, mu)
    samples = synth.eq9_samples(0.2, X.shape, ranks, True) if prob != "none" else None
    Qs, core, info = tr.tucker_rand_sthosvd(X, ranks, 10, 1, prob, samples, 5, diag="norms")
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) == 0
    for Q in Qs:
        Qd = Q.double()
        assert float(torch.linalg.matrix_norm(Qd.t() @ Qd - torch.eye(mu, dtype=torch.float64,
                                                                     device=Q.device))) < 1e-5
    B = core.double()
    for n, Q in enumerate(Qs):
        B = torch.movedim(torch.tensordot(Q.double(), B, dims=([1], [n])), 0, n)
    A = X.double()
    re = float(torch.linalg.vector_norm(A - B) / torch.linalg.vector_norm(A))
    assert abs(float(_np(info["norms"])[2]) - re) <= 3e-7, (re, float(_np(info["norms"])[2]))
    if prob == "none" and mu == 50:
        # the U(0,1) core leaves a rank-50 truncation of the 100^3 signal at RE ~0.47
        assert 0.3 < re < 0.6
    elif prob == "none":
        # rank 100 captures the signal: the noise level gamma = 1e-3 remains
        assert re < 2e-3
    else:
        # uniform samples of the ST-HOSVD intermediates miss its few dominant
        # columns with a probability that depends on the draw (the later modes
        # keep one column of the mean component in mu_1 mu_2 ... columns), so
        # the RE varies with the seed; it is checked against the outputs only
        assert re < 1.0


def test_tendiag_200cube_against_oracle():
    """Fifty equal leading singular values: individual columns inside the
    cluster are set by the sketch alone, so only subspaces (projector
    distance within max(1e-4, 1e2 u64 kappa_n), carried through the modes)
    and RE (1e-7) are compared."""
    v = [1.0 if i < 50 else float(i - 49) ** -2 for i in range(1, 201)]
    A = _np(synth.tendiag_noise_device((200, 200, 200), v, 1e-3, 13))
    ranks = (52, 52, 52)
    Qs, core, info = tr.tucker_rand_sthosvd(tr.to_device(A), ranks, 10, 1, seed=6,
                                            diag="norms")
    torch.cuda.synchronize()
    assert int(_np(info["status"])[0]) == 0
    Qg = [_np(Q).astype(np.float64) for Q in Qs]
    Qo, co, infos = oracle.rand_sthosvd(A, ranks, 10, 1, seed=6)
    bar = 1e-4
    for n in range(3):
        sig = infos[n]["sigma"]
        bar = max(bar, 1e2 * 2.0 ** -53 * sig[0] / max(sig[51] - sig[52], 1e-300))
        d = max(np.linalg.norm(Qg[n] - Qo[n] @ (Qo[n].T @ Qg[n]), 2),
                np.linalg.norm(Qo[n] - Qg[n] @ (Qg[n].T @ Qo[n]), 2))
        assert d <= bar, (n, d, bar)
    re_g = oracle.relative_error(A, _np(core).astype(np.float64), Qg)
    re_o = oracle.relative_error(A, co, Qo)
    assert abs(re_g - re_o) <= 1e-7, (re_g, re_o)
