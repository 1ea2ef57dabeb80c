"""Low-precision power-scheme products, emulated in numpy.

TEST INFRASTRUCTURE (see the package docstring).  This is not a step of the
paper: the paper computes every product in working precision.  It restates
the reduced-precision scheme of the library (products with bfloat16 or FP8
operands and float32 accumulation, float64 everywhere else) from the number
formats' definitions, so that the device results can be checked element by
element; the products and sums here are float64, so the two agree to float32
accumulation error.

Number formats (round to nearest, ties to even, from the float32 value):

* bfloat16: 8 exponent bits, 7 fraction bits -- the float32 value with its low
  16 bits rounded away.
* FP8 e4m3 in the OCP "e4m3fn" form: exponent bias 7, 3 fraction bits, no
  infinities; normal values (1 + f/8) 2^(e - 7) for e = 1..15 (for e = 15
  only f < 7, so the largest value is 448), subnormal values (f/8) 2^-6.
  Magnitudes beyond 448 saturate to 448 before rounding; NaN stays NaN.

Scaling (FP8 only; every scale is 1 for bfloat16).  For one power step
C <- M D M^T C on an I x J matrix M (a tensor unfolding, or the gathered
sample matrix C' with D = diag(scale_t^2)):

* C is rounded per column: tau_k = max_i |C(i, k)| / 448, Chat = e4m3(C / tau).
* A tensor unfolding is rounded with one scale: alpha = max |M| / 448,
  Mhat = e4m3(M * (448 / max |M|)), and D = alpha^2 I.
* The sample matrix is rounded per column when it is gathered:
  sigma_t = max_i |C'(i, t)| / 448, C'hat = e4m3(C' / sigma), and
  D = diag(scale_t^2 sigma_t^2).
* The columns are taken in blocks b of 32 consecutive columns.  For each
  block, W_b = D_b Mhat_b^T Chat diag(tau) (32 x s, float32), and
  C_new = sum over b of Mhat_b (hi_b + lo_b) with hi_b = bf16(W_b) and
  lo_b = bf16(W_b - hi_b): the slab enters the second product as a pair of
  bfloat16 matrices (about 16 significant bits), and Mhat in bfloat16, which
  holds every bfloat16 and every e4m3 value exactly.

For q > 1 the power scheme runs in its R-accumulated form: Z_0 R_0 = G (with
Z_0 = G and R_0 = I when s <= I / 2, where the Gaussian G is well
conditioned) and Z_i R_i = M D M^T Z_{i-1} (i = 1..q), where Z_i is the
orthonormal QR factor of the iterate with the canonical signs and
R_i = Z_i^T (M D M^T Z_{i-1}), and C_n = Z_q Rbar with Rbar = R_q ... R_0, equal to (M D M^T)^q G in exact
arithmetic.  Only orthonormal iterates (or that well-conditioned G) are
rounded to the operand format, so directions far below the leading one
survive the rounding.

Scale arithmetic follows the device in float32: tau and sigma are
max / 448 and the rounded value is x / scale; the tensor is multiplied by
448 / max.
"""
from __future__ import annotations

import numpy as np

from .tucker import canonical_signs, gaussian_matrix, leading_left_singular_vectors, unfold

FP8_MAX = 448.0
BLOCK = 32


def round_bf16(x) -> np.ndarray:
    """bfloat16 value of float32(x), as float64 (round to nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def _e4m3_values() -> np.ndarray:
    """All non-negative finite e4m3fn values, increasing (code = index)."""
    vals = [f / 8.0 * 2.0 ** -6 for f in range(8)]           # e = 0: subnormal
    for e in range(1, 16):
        for f in range(8):
            if e == 15 and f == 7:
                break                                        # that code is NaN
            vals.append((1.0 + f / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


E4M3_VALUES = _e4m3_values()


def round_e4m3(x) -> np.ndarray:
    """e4m3fn value of float32(x), as float64: saturate to +-448, then round
    to the nearest value, ties to the even code."""
    f = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.minimum(np.abs(f), FP8_MAX)
    hi = np.searchsorted(E4M3_VALUES, a, side="left")       # first value >= a
    hi = np.minimum(hi, len(E4M3_VALUES) - 1)
    lo = np.maximum(hi - 1, 0)
    vlo, vhi = E4M3_VALUES[lo], E4M3_VALUES[hi]
    dlo, dhi = a - vlo, vhi - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(a == vhi, hi, np.where(pick_hi, hi, lo))
    out = np.copysign(E4M3_VALUES[code], f)
    return np.where(np.isnan(f), np.nan, out)


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def quantize_columns(C: np.ndarray, prec: str):
    """(Chat, tau): column-scaled rounding of C (float64 values of the format)."""
    C32 = _f32(C)
    if prec == "bf16":
        return round_bf16(C32), np.ones(C.shape[1])
    mx = np.max(np.abs(C32), axis=0)
    tau = np.where(mx > 0, _f32(mx) / np.float32(FP8_MAX), np.float32(1.0)).astype(np.float32)
    return round_e4m3(C32 / tau[None, :]), tau.astype(np.float64)


def quantize_tensor(M: np.ndarray, prec: str):
    """(Mhat, d0): the unfolding rounded with one scale, and D = d0 I."""
    M32 = _f32(M)
    if prec == "bf16":
        return round_bf16(M32), 1.0
    mx = np.float32(np.max(np.abs(M32)))
    if mx == 0:
        return round_e4m3(M32), 1.0
    inv = np.float32(FP8_MAX) / mx
    alpha = mx / np.float32(FP8_MAX)
    return round_e4m3(M32 * inv), float(np.float32(alpha * alpha))


def quantize_samples(Cp_unscaled: np.ndarray, scale: np.ndarray, prec: str):
    """(C'hat, d): the gathered columns A_(n)(:, xi_t) rounded per column, and
    the column weights d_t = scale_t^2 sigma_t^2 (float32)."""
    A32 = _f32(Cp_unscaled)
    s2 = np.asarray(scale, dtype=np.float64) ** 2
    if prec == "bf16":
        return round_bf16(A32), _f32(s2).astype(np.float64)
    mx = np.max(np.abs(A32), axis=0)
    sig = np.where(mx > 0, mx / np.float32(FP8_MAX), np.float32(1.0)).astype(np.float32)
    d = _f32(s2 * sig.astype(np.float64) ** 2).astype(np.float64)
    return round_e4m3(A32 / sig[None, :]), d


def power_step(Mhat: np.ndarray, d: np.ndarray, C: np.ndarray, prec: str) -> np.ndarray:
    """One low-precision power step C <- Mhat D Mhat^T C (the block scheme above)."""
    Chat, tau = quantize_columns(C, prec)
    I, J = Mhat.shape
    out = np.zeros((I, C.shape[1]))
    for b0 in range(0, J, BLOCK):
        Mb = Mhat[:, b0:b0 + BLOCK]
        W = _f32((Mb.T @ Chat) * tau[None, :] * d[b0:b0 + BLOCK, None])
        hi = round_bf16(W)
        lo = round_bf16(_f32(W - hi))
        out += Mb @ (hi + lo)
    return out


def power_sketch_lp(X: np.ndarray, n: int, s: int, q: int, prec: str, seed: int,
                    xi=None, scale=None) -> np.ndarray:
    """C_n = (M D M^T)^q G_n in low precision for mode n of tensor X.

    Without ``xi``: M is the unfolding A_(n) (Alg. 1).  With ``xi``/``scale``
    (from ``oracle.randsample``): M is the sample matrix C'_n = A_(n) S_n
    (Alg. 4), rounded per column.
    """
    if prec not in ("bf16", "fp8e4m3"):
        raise ValueError(prec)
    An = unfold(np.asarray(X), n)
    I = An.shape[0]
    if xi is None:
        Mhat, d0 = quantize_tensor(An, prec)
        d = np.full(An.shape[1], d0)
    else:
        Mhat, d = quantize_samples(An[:, xi], scale, prec)
    G = gaussian_matrix(I, s, n, seed)
    if q == 1:
        return power_step(Mhat, d, G, prec)
    if 2 * s <= I:
        # a well-conditioned Gaussian start is rounded as it is: Z_0 = G, R_0 = I
        Z, Rbar = G, np.eye(s)
    else:
        Z, Rbar = _orth(G)
    for _ in range(q):
        Z, R = _orth(power_step(Mhat, d, Z, prec))
        Rbar = R @ Rbar
    return Z @ Rbar


def _orth(Y: np.ndarray):
    """(Z, R) with Z the orthonormal factor of the QR factorization of Y
    (canonical signs) and R = Z^T Y, so that Y = Z R."""
    Q, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64))
    Z = canonical_signs(Q)
    return Z, Z.T @ Y


def range_finder_lp(X, n: int, mu: int, K: int, q: int, prec: str, seed: int,
                    xi=None, scale=None):
    """(Q_n, C_n, sigma): the leading left singular vectors of the
    low-precision sketch (float64 SVD, canonical signs)."""
    I = np.asarray(X).shape[n]
    s = min(mu + K, I)
    C = power_sketch_lp(X, n, s, q, prec, seed, xi, scale)
    Q, sig = leading_left_singular_vectors(C, mu)
    return Q, C, sig
