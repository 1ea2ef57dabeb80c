"""Plain, slow FP64 oracle of randomized T-HOSVD and ST-HOSVD with the power
scheme and approximate matrix multiplication (Che, Wei, Yan, "Efficient
algorithms for Tucker decomposition via approximate matrix multiplication").

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import or call this package.  It shares no
code, header, table or helper with the HIP library, and the library never
calls it.

Every step is written from its definition in the paper, in the paper's order
and notation, with numpy (float64) as the only arithmetic:

* unfolding A_(n) and mode-n product x_n (Section 2);
* Alg. 1 / Alg. 2: C_n = (A_(n) A_(n)^T)^q G_n computed with Strategy A of the
  Remark after Alg. 1 (alternate A_(n)^T C and A_(n) C'), no re-orthonormalisation
  between power steps;
* Alg. 3 (BasicMatrixMultiplication) inside Alg. 4 / Alg. 5:
  C'_n = A_(n) S_n with S_n ~ RANDSAMPLE(T_n, p_n), then C_n = (C'_n C'_n^T)^q G_n;
* Q_n = first mu_n left singular vectors of C_n (Remark after Alg. 5);
* T-HOSVD core G = A x_1 Q_1^T ... x_N Q_N^T (Alg. 1 / Alg. 4);
  ST-HOSVD update A <- A x_n Q_n^T after each mode (Alg. 2 / Alg. 5);
* the related forms (Alg. 6 for Alg. 1, Alg. 7 for Alg. 2, and by the Remark
  closing that subsection the same change to Alg. 4 / Alg. 5): a thin QR
  C_n = P_n R, then U_n = the mu_n leading left singular vectors of
  P_n^T A_(n), and Q_n = P_n U_n;
* relative error RE of Eq. (8).

Readings where the paper is silent (all listed in the design notes):

* Random numbers.  The paper only says "standard Gaussian matrix" and
  "RANDSAMPLE".  Both come from Philox4x64-10 (``oracle.philox``) with key
  (seed, 0).  Gaussian G_n (I_n x s_n, column-major element e = i + I_n*c):
  counter (e // 4, n, 0, 0); output words (0,1) and (2,3) are Box-Muller pairs
  u1 = ((r_a >> 11) + 1) * 2^-53, u2 = (r_b >> 11) * 2^-53,
  z_a = sqrt(-2 ln u1) cos(2 pi u2), z_b = sqrt(-2 ln u1) sin(2 pi u2).
  Sample draw t: counter (t // 2, n, 1, 0), words (2(t%2), 2(t%2)+1) = (h, l).
  Mode index n is 0-based.
* Sketch width s_n = min(mu_n + K, I_n).
* Nearly-optimal probabilities (Remark after Alg. 3, the beta = 1 form
  p_j = ||A_(n)(:,j)||^2 / ||A_(n)||_F^2, which is the optimal choice for the
  product A_(n) A_(n)^T).  Column norms are accumulated row by row in float64
  in increasing row order.  They are quantised, without any order-dependent sum,
  to integer weights w_j = floor((n_j / max_k n_k) * 2^k), k = 60 - ceil(log2 J),
  raised to 1 for every non-zero column; p~_j = w_j / W with W = sum w_j (exact).
  Uniform probabilities use w_j = 1.
* Draw t picks xi_t = min{ j : cdf_j > x_t } with cdf the inclusive prefix sum
  of w and x_t = floor((h*2^64 + l) * W / 2^128) computed exactly.
* Rescale 1/sqrt(T p~_xi) evaluated as sqrt((W / w_xi) / T) in three IEEE
  double operations in that order.
* If T_n > J_n the mode is computed exactly (C'_n := A_(n)); Alg. 3 requires
  T <= J.
* Sign of each singular vector: the entry of largest magnitude (lowest row on
  ties) is made positive.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np

from .philox import philox4x64

TAG_GAUSS = 0
TAG_SAMPLE = 1
TWO_PI = 6.283185307179586  # the double nearest 2*pi (exactly 2 * math.pi)

PROB_NONE = "none"
PROB_NEARLY_OPTIMAL = "nearly_optimal"
PROB_UNIFORM = "uniform"
PROBS = (PROB_NONE, PROB_NEARLY_OPTIMAL, PROB_UNIFORM)


# --------------------------------------------------------------------------
# Section 2: unfolding, mode-n product, norms
# --------------------------------------------------------------------------

def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding A_(n) (Section 2), 0-based modes.

    Element (i_1..i_N) goes to row i_n and column
    j = sum_{k != n} i_k prod_{m < k, m != n} I_m  (0-based form of the paper's map).
    """
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1, order="F")


def fold(M: np.ndarray, n: int, shape: Sequence[int]) -> np.ndarray:
    """Inverse of ``unfold`` for a tensor of the given shape."""
    shape = tuple(shape)
    moved = (shape[n],) + shape[:n] + shape[n + 1:]
    return np.moveaxis(M.reshape(moved, order="F"), 0, n)


def mode_product(X: np.ndarray, B: np.ndarray, n: int) -> np.ndarray:
    """X x_n B for B of size J x I_n (Section 2): C_(n) = B X_(n)."""
    shape = list(X.shape)
    shape[n] = B.shape[0]
    return fold(B @ unfold(X, n), n, shape)


def frobenius(X: np.ndarray) -> float:
    """||X||_F = sqrt(<X, X>) (Section 2)."""
    return float(np.sqrt(np.sum(np.asarray(X, dtype=np.float64) ** 2)))


def column_sq_norms(An: np.ndarray) -> np.ndarray:
    """n_j = ||A_(n)(:, j)||_2^2, accumulated over rows i = 0, 1, ... in float64."""
    An = np.asarray(An, dtype=np.float64)
    acc = np.zeros(An.shape[1])
    for i in range(An.shape[0]):
        acc = acc + An[i, :] * An[i, :]
    return acc


# --------------------------------------------------------------------------
# Random inputs of the method: Gaussian G_n and RANDSAMPLE (Section 3.2)
# --------------------------------------------------------------------------

def gaussian_matrix(I: int, s: int, mode: int, seed: int) -> np.ndarray:
    """Standard Gaussian matrix G_n in R^{I x s} (Alg. 1, step 2; Section 5.1)."""
    total = I * s
    G = np.zeros(total)
    for b in range((total + 3) // 4):
        r = philox4x64((b, mode, TAG_GAUSS, 0), (seed, 0))
        for pair in range(2):
            ra, rb = r[2 * pair], r[2 * pair + 1]
            u1 = float((ra >> 11) + 1) * 2.0 ** -53
            u2 = float(rb >> 11) * 2.0 ** -53
            rho = math.sqrt(-2.0 * math.log(u1))
            theta = TWO_PI * u2
            e = 4 * b + 2 * pair
            if e < total:
                G[e] = rho * math.cos(theta)
            if e + 1 < total:
                G[e + 1] = rho * math.sin(theta)
    return G.reshape(I, s, order="F")


def ceil_log2(J: int) -> int:
    """ceil(log2 J) for J >= 1, in exact integer arithmetic."""
    return (int(J) - 1).bit_length()


def sampling_weights(norms: Optional[np.ndarray], J: int, prob: str) -> np.ndarray:
    """Integer weights w_j defining p~_j = w_j / sum(w) (Remark after Alg. 3)."""
    if prob == PROB_UNIFORM:
        return np.ones(J, dtype=np.uint64)
    if prob != PROB_NEARLY_OPTIMAL:
        raise ValueError(prob)
    norms = np.asarray(norms, dtype=np.float64)
    if norms.shape != (J,) or not np.all(np.isfinite(norms)):
        raise FloatingPointError("column norms must be finite")
    M = float(norms.max())
    if M <= 0.0:
        raise FloatingPointError("all columns are zero: no sampling distribution")
    k = 60 - ceil_log2(J)
    w = np.floor((norms / M) * (2.0 ** k)).astype(np.uint64)
    w = np.where(norms > 0.0, np.maximum(w, np.uint64(1)), np.uint64(0))
    return w.astype(np.uint64)


def draw_columns(w: np.ndarray, T: int, seed: int, mode: int):
    """xi_t ~ MULTINOMIAL(p~), t < T, and s_t = 1/sqrt(T p~_xi) (RANDSAMPLE, Section 3.2).

    Returns (xi, scale, W) with xi int64[T] (0-based column indices).
    """
    cdf = np.cumsum(w, dtype=np.uint64)
    W = int(cdf[-1])
    xi = np.zeros(T, dtype=np.int64)
    scale = np.zeros(T)
    for t in range(T):
        r = philox4x64((t // 2, mode, TAG_SAMPLE, 0), (seed, 0))
        h, l = r[2 * (t % 2)], r[2 * (t % 2) + 1]
        x = (W * h + ((W * l) >> 64)) >> 64
        j = int(np.searchsorted(cdf, np.uint64(x), side="right"))
        xi[t] = j
        scale[t] = math.sqrt((float(W) / float(int(w[j]))) / float(T))
    return xi, scale, W


def randsample(norms, J: int, T: int, prob: str, seed: int, mode: int):
    """S ~ RANDSAMPLE(T, p) as (xi, scale): S[xi_t, t] = scale_t (Section 3.2)."""
    w = sampling_weights(norms, J, prob)
    xi, scale, W = draw_columns(w, T, seed, mode)
    return xi, scale, w, W


# --------------------------------------------------------------------------
# Per-mode range finder (Alg. 1 steps 2-5, Alg. 4 steps 2-7)
# --------------------------------------------------------------------------

def power_sketch(M: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """C = (M M^T)^q G by Strategy A (Remark after Alg. 1)."""
    C = np.array(G, dtype=np.float64)
    for _ in range(q):
        Cp = M.T @ C
        C = M @ Cp
    return C


def power_sketch_stabilised(M: np.ndarray, G: np.ndarray, q: int):
    """(Y_q, Rbar) with Y_q Rbar = (M M^T)^q G, QR after every power step.

    Y_0 R_0 = qr(G); Y_i R_i = qr(M M^T Y_{i-1}); Rbar = R_q ... R_0.  Equal to
    ``power_sketch`` in exact arithmetic; kept as a numerically safer variant.
    """
    Y, R = np.linalg.qr(np.array(G, dtype=np.float64))
    Rbar = R
    for _ in range(q):
        Y, R = np.linalg.qr(M @ (M.T @ Y))
        Rbar = R @ Rbar
    return Y, Rbar


def canonical_signs(Q: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (lowest row on ties)."""
    Q = np.array(Q, dtype=np.float64)
    for c in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, c])))
        if Q[i, c] < 0:
            Q[:, c] = -Q[:, c]
    return Q


def leading_left_singular_vectors(C: np.ndarray, mu: int):
    """Q_n = U_n(:, 1:mu_n) of the SVD C_n = U_n S_n V_n^T (Remark after Alg. 5)."""
    U, sig, _ = np.linalg.svd(C, full_matrices=False)
    return canonical_signs(U[:, :mu]), sig


def check_mode_args(I: int, J: int, mu: int, K: int, q: int, prob: str, T):
    if prob not in PROBS:
        raise ValueError(f"unknown probability type {prob!r}")
    if not (1 <= mu <= min(I, J)):
        raise ValueError(f"rank {mu} outside [1, min(I_n={I}, J_n={J})]")
    if K < 0 or q < 1:
        raise ValueError("need K >= 0 and q >= 1")
    if prob != PROB_NONE and (T is None or T < 1):
        raise ValueError("sampling needs T_n >= 1")


def related_factor(An: np.ndarray, C: np.ndarray, mu: int):
    """Q_n of the related forms (Alg. 6 / Alg. 7 steps 5-7): thin QR
    C_n = P_n R (Householder, numpy), U_n = the mu leading left singular
    vectors of C'_n = P_n^T A_(n), Q_n = P_n U_n (canonical signs).  Returns
    (Q_n, P_n, singular values of C'_n)."""
    P, _ = np.linalg.qr(C)
    Cp = P.T @ An
    U, sig, _ = np.linalg.svd(Cp, full_matrices=False)
    return canonical_signs(P @ U[:, :mu]), P, sig


def range_finder(X: np.ndarray, n: int, mu: int, K: int, q: int, prob: str,
                 T: Optional[int], seed: int, stabilised: bool = False,
                 related: bool = False):
    """Q_n for mode n of the current tensor X, plus intermediates for tests.

    prob == "none": Alg. 1 steps 2-5 (C_n = (A_(n) A_(n)^T)^q G_n).
    otherwise:      Alg. 4 steps 2-7 (C'_n = A_(n) S_n, C_n = (C'_n C'_n^T)^q G_n).
    related:        Q_n from C_n by the related form (``related_factor``).
    """
    An = unfold(np.asarray(X, dtype=np.float64), n)
    I, J = An.shape
    check_mode_args(I, J, mu, K, q, prob, T)
    s = min(mu + K, I)
    info = {"I": I, "J": J, "s": s, "exact": True}
    if prob == PROB_NONE or T > J:
        M = An
    else:
        norms = column_sq_norms(An) if prob == PROB_NEARLY_OPTIMAL else None
        xi, scale, w, W = randsample(norms, J, T, prob, seed, n)
        M = An[:, xi] * scale[None, :]           # C'_n = A_(n) S_n
        info.update(exact=False, norms=norms, w=w, W=W, xi=xi, scale=scale, Cp=M)
    G = gaussian_matrix(I, s, n, seed)
    info["G"] = G
    if stabilised:
        Y, Rbar = power_sketch_stabilised(M, G, q)
        Up, sig, _ = np.linalg.svd(Rbar)
        Q = canonical_signs(Y @ Up[:, :mu])
        info.update(C=Y @ Rbar, sigma=sig)
    else:
        C = power_sketch(M, G, q)
        Q, sig = leading_left_singular_vectors(C, mu)
        info.update(C=C, sigma=sig)
    if related:
        Q, P, sig_cp = related_factor(An, info["C"], mu)
        info.update(P=P, sigma_related=sig_cp)
    return Q, info


# --------------------------------------------------------------------------
# Drivers
# --------------------------------------------------------------------------

def _as_f64(A) -> np.ndarray:
    return np.asarray(A, dtype=np.float64)


def _per_mode(v, N, name):
    if v is None:
        return [None] * N
    v = list(v)
    if len(v) != N:
        raise ValueError(f"{name} needs {N} entries")
    return v


def rand_thosvd(A, ranks, K: int, q: int, prob: str = PROB_NONE, samples=None,
                seed: int = 0, stabilised: bool = False, related: bool = False):
    """Alg. 1 (prob == "none") or Alg. 4 (sampled), or with ``related`` their
    related form (Alg. 6): returns (Q list, core, infos)."""
    X = _as_f64(A)
    N = X.ndim
    ranks = _per_mode(ranks, N, "ranks")
    samples = _per_mode(samples, N, "samples")
    Qs: List[np.ndarray] = []
    infos = []
    for n in range(N):
        Q, info = range_finder(X, n, ranks[n], K, q, prob, samples[n], seed,
                               stabilised, related)
        Qs.append(Q)
        infos.append(info)
    core = X
    for n in range(N):
        core = mode_product(core, Qs[n].T, n)
    return Qs, core, infos


def rand_sthosvd(A, ranks, K: int, q: int, prob: str = PROB_NONE, samples=None,
                 seed: int = 0, stabilised: bool = False, related: bool = False):
    """Alg. 2 (prob == "none") or Alg. 5 (sampled), or with ``related`` their
    related form (Alg. 7): returns (Q list, core, infos)."""
    X = _as_f64(A)
    N = X.ndim
    ranks = _per_mode(ranks, N, "ranks")
    samples = _per_mode(samples, N, "samples")
    Qs: List[np.ndarray] = []
    infos = []
    for n in range(N):
        Q, info = range_finder(X, n, ranks[n], K, q, prob, samples[n], seed,
                               stabilised, related)
        info["X_before"] = X
        X = mode_product(X, Q.T, n)              # A <- A x_n Q_n^T
        Qs.append(Q)
        infos.append(info)
    return Qs, X, infos


def reconstruct(core: np.ndarray, Qs: Sequence[np.ndarray]) -> np.ndarray:
    """A^ = G x_1 Q_1 x_2 Q_2 ... x_N Q_N (Eq. (1) with orthonormal factors)."""
    X = _as_f64(core)
    for n, Q in enumerate(Qs):
        X = mode_product(X, Q, n)
    return X


def relative_error(A, core, Qs) -> float:
    """RE = ||A - A^||_F / ||A||_F, Eq. (8)."""
    A = _as_f64(A)
    return frobenius(A - reconstruct(core, Qs)) / frobenius(A)


# --------------------------------------------------------------------------
# Fixed-precision problem (Problem 2, Section 7): ranks chosen for a tolerance
# --------------------------------------------------------------------------

def choose_rank(lam: np.ndarray, x2: float, budget: float, mu_max: int) -> int:
    """Smallest mu in [1, mu_max] whose residual x2 - sum_{k <= mu} lam_k is at
    most ``budget`` (mu_max when none is).  lam: squared singular values of
    P_n^T X_(n), descending; x2 = ||X||_F^2."""
    for mu in range(1, mu_max + 1):
        if x2 - float(np.sum(lam[:mu])) <= budget:
            return mu
    return mu_max


def rand_tucker_adaptive(A, eps: float, max_ranks, K: int, q: int, prob: str = PROB_NONE,
                         samples=None, seed: int = 0, sthosvd: bool = True):
    """Problem 2 (find mu_n and orthonormal Q_n with ||A - A^||_F <= eps).

    The paper poses it without an algorithm; this is the rule the library
    implements.  Each mode is computed by the related form (Alg. 6 / Alg. 7),
    whose P_n^T X_(n) gives the residual of every candidate rank exactly:
    ||X x_n (I - Q_n Q_n^T)||_F^2 = ||X||_F^2 - sum_{k <= mu} sigma_k(P_n^T X_(n))^2
    for Q_n = P_n U_n(:, 1:mu).  mu_n is the smallest rank (at most
    min(max_ranks[n], J_n)) whose residual fits the mode's budget:
    T-HOSVD eps^2 / N per mode (Eq. (5)); ST-HOSVD the budget left by the
    modes before, split evenly over the remaining ones (Eq. (23)).  Returns
    (Q list, core, chosen ranks, bound) with bound = sqrt(sum of the chosen
    residuals) >= ||A - A^||_F (Eq. (5) / Eq. (23)).  The residuals are float64
    differences with an absolute error of ~u ||A||^2, so tolerances below
    ~sqrt(u) ||A|| cannot be certified."""
    X = _as_f64(A)
    N = X.ndim
    max_ranks = _per_mode(max_ranks, N, "max_ranks")
    samples = _per_mode(samples, N, "samples")
    eps2 = float(eps) ** 2
    used = 0.0
    Qs, mus = [], []
    cur = X
    for n in range(N):
        src = cur if sthosvd else X
        An = unfold(src, n)
        # the sketch width follows the largest allowed rank, s_n =
        # min(max_rank_n + K, I_n), whatever ranks the earlier modes chose
        # (range_finder with rank 1 and oversampling s_n - 1 draws that sketch)
        s_n = min(max_ranks[n] + K, An.shape[0])
        _, info = range_finder(src, n, 1, s_n - 1, q, prob, samples[n], seed)
        P, _ = np.linalg.qr(info["C"])
        U, sig, _ = np.linalg.svd(P.T @ An, full_matrices=False)
        lam = sig ** 2
        x2 = frobenius(src) ** 2
        budget = (eps2 - used) / (N - n) if sthosvd else eps2 / N
        mu = choose_rank(lam, x2, budget, min(max_ranks[n], An.shape[1], len(lam)))
        used += max(x2 - float(np.sum(lam[:mu])), 0.0)
        Q = canonical_signs(P @ U[:, :mu])
        Qs.append(Q)
        mus.append(mu)
        if sthosvd:
            cur = mode_product(cur, Q.T, n)
    core = cur
    if not sthosvd:
        for n in range(N):
            core = mode_product(core, Qs[n].T, n)
    return Qs, core, mus, math.sqrt(used)
