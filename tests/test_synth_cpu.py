"""Host checks of the paper-workload generators (no GPU: torch on the CPU).

* the device-side Eq. (9) builder gives the same signal as the numpy builder
  (same draws; the noise comes from another generator, so gamma = 0 here);
* the Section 6.3 builder's unfoldings have exactly the singular values v;
* the noise is scaled to gamma ||B||_F / sqrt(prod I_n);
* T_n for Alg. 4 / Alg. 5 follows the Section 4.3 rule.
"""
import math

import numpy as np
import torch

import oracle
import synth


def test_device_tucker_matches_numpy_signal():
    X = synth.tucker_noise_device((20, 16, 12), (4, 3, 2), 0.0, 5, device="cpu",
                                  dtype=torch.float64)
    A = synth.low_rank_plus_noise((20, 16, 12), (4, 3, 2), 0.0, 5, core="uniform")
    assert X.stride() == (1, 20, 320)
    assert np.abs(X.numpy() - A).max() <= 1e-14
    X4 = synth.tucker_noise_device((6, 5, 4, 3), (2, 2, 2, 2), 0.0, 7, device="cpu",
                                   dtype=torch.float64, core="gauss")
    A4 = synth.low_rank_plus_noise((6, 5, 4, 3), (2, 2, 2, 2), 0.0, 7)
    assert np.abs(X4.numpy() - A4).max() <= 1e-14


def test_device_tendiag_singular_values():
    v = [1.0, 0.5, 0.25, 0.1]
    T = synth.tendiag_noise_device((10, 9, 8), v, 0.0, 3, device="cpu", dtype=torch.float64)
    for n in range(3):
        sv = np.linalg.svd(oracle.unfold(T.numpy(), n), compute_uv=False)
        assert np.allclose(sv[:4], v, atol=1e-13) and np.all(sv[4:] < 1e-13)


def test_device_noise_level():
    B = synth.tucker_noise_device((30, 20, 10), (3, 3, 3), 0.0, 9, device="cpu",
                                  dtype=torch.float64)
    A = synth.tucker_noise_device((30, 20, 10), (3, 3, 3), 0.1, 9, device="cpu",
                                  dtype=torch.float64)
    ratio = float(torch.linalg.vector_norm(A - B) / torch.linalg.vector_norm(B))
    assert abs(ratio - 0.1) < 0.01


def test_eq9_samples_rule():
    assert synth.eq9_samples(0.2, (600, 600, 600), (50, 50, 50), False) == (72000,) * 3
    assert synth.eq9_samples(0.2, (600, 600, 600), (50, 50, 50), True) == (72000, 6000, 500)
    assert synth.eq9_samples(0.01, (200,) * 4, (20,) * 4, True) == (
        80000, math.ceil(0.01 * 20 * 200 * 200), math.ceil(0.01 * 20 * 20 * 200),
        math.ceil(0.01 * 20 ** 3))


def test_csc_mode1_round_trip_and_sparse_generator():
    X = synth.sparse_cp_device((30, 20, 10), 30, 0.2, 1000, 3, device="cpu", dtype=torch.float64)
    A = X.numpy()
    # each factor vector has ceil(0.2 I_n) nonzeros, so the tensor is sparse
    assert 0.0 < np.mean(A != 0) < 0.5
    colptr, rowidx, vals = synth.csc_mode1(X)
    assert colptr[0] == 0 and colptr[-1] == vals.numel() == int(np.count_nonzero(A))
    D = np.zeros((30, 200))
    cp, ri, v = colptr.numpy(), rowidx.numpy(), vals.numpy()
    for j in range(200):
        rows = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(rows) > 0)
        D[rows, j] = v[cp[j]:cp[j + 1]]
    assert np.array_equal(D, A.reshape(30, 200, order="F"))
