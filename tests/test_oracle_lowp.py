"""Pins of the low-precision emulation (oracle/lowp.py).

* the two roundings against torch's own casts (bfloat16, float8_e4m3fn), a
  library routine written independently of the emulation, on random values
  spanning the formats' ranges and on hand-picked boundary cases;
* the e4m3fn value table against the format's defining numbers (127
  non-negative finite values, largest 448, smallest normal 2^-6, smallest
  subnormal 2^-9);
* one power step on data whose scaled values are small integers, where every
  rounding is exact: the emulated step must equal the exact product
  M D M^T C computed in integers (a lost scale tau, alpha^2 or weight d, or a
  wrong block boundary, changes the result);
* the size of the rounding effect: a bfloat16 / e4m3 sketch differs from the
  float64 sketch by about the formats' unit roundoff, and its leading
  subspace matches the float64 one.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import lowp


def _values(n=20000, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) * 10.0 ** rng.uniform(-12, 3, n)
    edge = [0.0, -0.0, 1.0, -1.0, 448.0, 447.9, 1.0625, 1.1875, 2.0 ** -9, 2.0 ** -10,
            1.5 * 2.0 ** -10, 2.0 ** -6, 240.0, 1.00390625, 1.01171875, 3.3e38, 1e-40]
    return np.concatenate([x, edge]).astype(np.float32)


def test_bf16_rounding_matches_torch():
    x = _values()
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_bf16(x), ref)
    # ties to even: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert lowp.round_bf16(np.float32(1.00390625)) == 1.0
    assert lowp.round_bf16(np.float32(1.01171875)) == 1.015625
    assert np.isnan(lowp.round_bf16(np.float32(np.nan)))


def test_e4m3_rounding_matches_torch():
    x = np.clip(_values(), -448.0, 448.0)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_e4m3(x), ref)


def test_e4m3_saturates_and_keeps_nan():
    out = lowp.round_e4m3(np.array([449.0, 500.0, 1e30, -1e30, -460.0], np.float32))
    assert np.array_equal(out, [448.0, 448.0, 448.0, -448.0, -448.0])
    assert np.isnan(lowp.round_e4m3(np.float32(np.nan)))


def test_e4m3_table():
    v = lowp.E4M3_VALUES
    assert len(v) == 127 and v[0] == 0.0 and v[-1] == 448.0
    assert v[1] == 2.0 ** -9 and v[8] == 2.0 ** -6
    assert np.all(np.diff(v) > 0)


@pytest.mark.parametrize("prec", ["bf16", "fp8e4m3"])
def test_power_step_exact_on_representable_data(prec):
    # integers in [-7, 7] with a 7 in every column: every scale is a power of
    # two (7 / 448 = 2^-6), every scaled value lies in the format, and the
    # slabs W are integers below 2^16 (exact as a bfloat16 pair)
    rng = np.random.default_rng(1)
    I, J, s = 24, 70, 5                      # J spans three blocks, the last ragged
    M = rng.integers(-7, 8, size=(I, J)).astype(np.float64)
    M[0, :] = 7.0
    C = rng.integers(-7, 8, size=(I, s)).astype(np.float64)
    C[1, :] = 7.0
    d = rng.integers(1, 4, size=J).astype(np.float64)
    if prec == "bf16":
        Mhat, d0 = lowp.quantize_tensor(M, prec)
        assert d0 == 1.0
    else:
        Mhat, d0 = lowp.quantize_tensor(M, prec)
        assert d0 == 2.0 ** -12             # alpha = 7 / 448 = 2^-6
        assert np.array_equal(Mhat, 64.0 * M)
    out = lowp.power_step(Mhat, d * d0, C, prec)
    exact = M @ (d[:, None] * (M.T @ C))
    assert np.array_equal(out, exact)


@pytest.mark.parametrize("prec,tol", [("bf16", 8e-3), ("fp8e4m3", 0.1)])
@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("K", [6, 10])
def test_sketch_error_is_format_sized(prec, tol, q, K):
    # K = 10 gives mode 3 (I = 20) s = 14 > I / 2: its q = 2 scheme starts from
    # an orthonormal basis of G; every other mode starts from G itself
    A = synth.low_rank_plus_noise((40, 30, 20), (4, 4, 4), 1e-3, 5, np.float32)
    A64 = A.astype(np.float64)
    for n in range(3):
        I = A.shape[n]
        s = min(4 + K, I)
        C = lowp.power_sketch_lp(A, n, s, q, prec, 7)
        Q, _ = oracle.leading_left_singular_vectors(C, 4)
        Ce = oracle.power_sketch(oracle.unfold(A64, n), oracle.gaussian_matrix(I, s, n, 7), q)
        Qe, _ = oracle.leading_left_singular_vectors(Ce, 4)
        # q = 2 too: the R-accumulated sketch Z_q Rbar is the plain product in
        # exact arithmetic, so it carries only the format's rounding
        assert np.linalg.norm(C - Ce) / np.linalg.norm(Ce) <= tol
        # the leading subspace: within the format's roundoff of the float64 one
        assert np.linalg.norm(Q @ Q.T - Qe @ Qe.T, 2) <= tol


def test_sampled_sketch_uses_sample_weights():
    # C' D C'^T with D = diag(scale^2): rounding C' per column must keep the
    # weights; the bfloat16 result is within roundoff of the float64 one
    A = synth.low_rank_plus_noise((30, 20, 10), (3, 3, 3), 1e-3, 2, np.float32)
    A64 = A.astype(np.float64)
    An = oracle.unfold(A64, 0)
    xi, scale, _, _ = oracle.randsample(oracle.column_sq_norms(An), An.shape[1], 64,
                                        "nearly_optimal", 3, 0)
    for prec, tol in (("bf16", 8e-3), ("fp8e4m3", 0.1)):
        C = lowp.power_sketch_lp(A, 0, 8, 1, prec, 3, xi, scale)
        Ce = oracle.power_sketch(An[:, xi] * scale[None, :], oracle.gaussian_matrix(30, 8, 0, 3), 1)
        assert np.linalg.norm(C - Ce) / np.linalg.norm(Ce) <= tol
