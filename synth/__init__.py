"""Seeded synthetic input tensors shaped like the paper's test problems.

This module only draws random numbers and assembles tensors of a known
structure; it holds none of the decomposition's arithmetic.  The oracle and the
GPU path both consume its arrays, and neither is imported here.

Constructions (all in float64 with ``numpy.random.default_rng(seed)``, rounded
once to the storage dtype at the very end):

* ``orth(X)``: the Q factor of a Householder QR of a Gaussian matrix, with the
  signs fixed so that diag(R) > 0 -- "an orthonormal basis for the column space
  of a standard Gaussian matrix" as in the Eq. (9) test tensor (Section 4.3).
* Tucker-form signal plus noise, Eq. (9): A = B + gamma*||B||_F/sqrt(prod I_n)*E,
  B = C x_1 U_1 ... x_N U_N, E iid N(0,1).  The paper's divisor sqrt(400^3) for
  a 600^3 tensor is read as sqrt(prod I_n), so that ||noise||_F ~ gamma*||B||_F.
* Superdiagonal core tendiag(v) (Section 6.3): every mode-n unfolding of the
  signal then has the singular values v exactly.
* Sum of separable Gaussian bumps (a smooth, image-like field).

Draw order is fixed: core (or bump amplitudes), then factors 1..N (or bump
centres and widths per mode), then noise.

Arrays are returned in column-major (Fortran) order: the first index is the
fastest, i.e. mode-1 fibers are contiguous, which is the layout the library and
the paper's unfolding (Section 2) use.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "orth", "tucker_signal", "tendiag", "add_noise", "Workload",
    "low_rank_plus_noise", "gaussian_bumps", "config", "CONFIGS",
    "serving_request", "serving_shape", "serving_request_device",
    "tucker_noise_device", "tendiag_noise_device", "eq9_samples",
    "sparse_cp_device", "csc_mode1",
]


def orth(X: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(X) (Householder QR, diag(R) > 0)."""
    Q, R = np.linalg.qr(X)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def tucker_signal(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """B = core x_1 U_1 x_2 U_2 ... x_N U_N, returned Fortran-ordered float64."""
    B = np.asarray(core, dtype=np.float64)
    for n, U in enumerate(factors):
        B = np.moveaxis(np.tensordot(U, B, axes=(1, n)), 0, n)
    return np.asfortranarray(B)


def tendiag(v: Sequence[float], order: int) -> np.ndarray:
    """Superdiagonal tensor with v on its diagonal (entries (k,k,...,k))."""
    r = len(v)
    C = np.zeros((r,) * order)
    for k in range(r):
        C[(k,) * order] = v[k]
    return C


def add_noise(B: np.ndarray, gamma: float, rng: np.random.Generator) -> np.ndarray:
    """A = B + gamma*||B||_F/sqrt(prod(I_n))*E with E iid N(0,1)."""
    if gamma == 0.0:
        return B
    scale = gamma * float(np.linalg.norm(B.ravel(order="K"))) / math.sqrt(B.size)
    E = rng.standard_normal(B.shape[::-1]).T  # Fortran-ordered draw, same stream
    B = B + scale * E
    return np.asfortranarray(B)


@dataclasses.dataclass
class Workload:
    """A generated tensor plus the decomposition parameters it is run with."""
    name: str
    A: np.ndarray                 # Fortran-ordered, storage dtype
    ranks: tuple
    oversample: int
    power: int
    algo: str                     # "thosvd" | "sthosvd"
    prob: str                     # "none" | "nearly_optimal" | "uniform"
    samples: Optional[tuple]      # T_n per mode (None if prob == "none")
    seed: int
    precision: str = "native"
    note: str = ""

    @property
    def dims(self) -> tuple:
        return tuple(self.A.shape)


def low_rank_plus_noise(dims, core_dims, gamma, seed, dtype=np.float64,
                        core="gauss", decay=None) -> np.ndarray:
    """Tucker-form signal plus relative Gaussian noise (Eq. (9) style).

    core="gauss": iid N(0,1) core; core="uniform": iid U(0,1) core (Eq. (9));
    core="tendiag": superdiagonal core with diagonal ``decay`` (Section 6.3).
    """
    rng = np.random.default_rng(seed)
    N = len(dims)
    if core == "gauss":
        C = rng.standard_normal(tuple(core_dims)[::-1]).T
    elif core == "uniform":
        C = rng.random(tuple(core_dims)[::-1]).T
    elif core == "tendiag":
        assert decay is not None and all(c == len(decay) for c in core_dims)
        C = tendiag(decay, N)
    else:
        raise ValueError(core)
    U = [orth(rng.standard_normal((dims[n], core_dims[n]))) for n in range(N)]
    if core == "tendiag":
        # Sum of r rank-one terms; built mode by mode to keep memory modest.
        B = _cp_sum(np.asarray(decay, dtype=np.float64), U)
    else:
        B = tucker_signal(C, U)
    A = add_noise(B, gamma, rng)
    return np.asfortranarray(A.astype(dtype))


def _cp_sum(weights: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """sum_b w_b * f1_b o f2_b o ... o fN_b, Fortran-ordered float64."""
    N = len(factors)
    # Build the Fortran-ordered result as a C-ordered array of reversed shape.
    rev = factors[::-1]
    letters = "abcdefgh"[:N]
    spec = ",".join(f"{letters[i]}z" for i in range(N)) + ",z->" + letters
    out = np.ascontiguousarray(np.einsum(spec, *rev, weights, optimize=True))
    return out.T  # shape (I_1..I_N), Fortran-contiguous view


def gaussian_bumps(dims, n_bumps, seed, dtype=np.float32, width=(4.0, 32.0),
                   nonneg=False) -> np.ndarray:
    """Sum of separable Gaussian bumps: A(i) = sum_b a_b prod_n exp(-(i_n-c)^2/(2w^2)).

    a_b ~ N(0,1) (|a_b| if nonneg), centres c_{b,n} ~ U[0, I_n), widths
    w_{b,n} ~ U[width]. One width per bump per mode.
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n_bumps)
    if nonneg:
        a = np.abs(a)
    F = []
    for I in dims:
        c = rng.random(n_bumps) * I
        w = width[0] + (width[1] - width[0]) * rng.random(n_bumps)
        i = np.arange(I, dtype=np.float64)[:, None]
        F.append(np.exp(-((i - c[None, :]) ** 2) / (2.0 * w[None, :] ** 2)))
    return np.asfortranarray(_cp_sum(a, F).astype(dtype))


def config(k: int, seed: int = 0) -> Workload:
    """The five benchmark configurations (1-based ``k``), synthesised.

    1: 64^3 float64, Gaussian core 5^3, noise 1e-3, Alg. 1 (T-HOSVD), exact.
    2: 400^3 float32, tendiag core 0.5^k (k<10), noise 1e-4, Alg. 5
       (ST-HOSVD + AMM), nearly-optimal probabilities, T_n = 4000.
    3: 100^4 float32, tendiag core (k+1)^-2 (k<20), noise 1e-3, q = 2.
    4: 512x512x256 float32, 50 Gaussian bumps, Alg. 4, uniform, T_n = 8000.
    """
    if k == 1:
        A = low_rank_plus_noise((64, 64, 64), (5, 5, 5), 1e-3, seed, np.float64)
        return Workload("c1_64cube_f64_thosvd", A, (5, 5, 5), 5, 1, "thosvd",
                        "none", None, seed)
    if k == 2:
        v = [0.5 ** i for i in range(10)]
        A = low_rank_plus_noise((400, 400, 400), (10, 10, 10), 1e-4, seed,
                                np.float32, core="tendiag", decay=v)
        return Workload("c2_400cube_f32_sthosvd_amm", A, (10, 10, 10), 10, 1,
                        "sthosvd", "nearly_optimal", (4000, 4000, 4000), seed)
    if k == 3:
        v = [(i + 1.0) ** -2 for i in range(20)]
        A = low_rank_plus_noise((100, 100, 100, 100), (20,) * 4, 1e-3, seed,
                                np.float32, core="tendiag", decay=v)
        return Workload("c3_100pow4_f32", A, (20,) * 4, 10, 2, "thosvd", "none",
                        None, seed)
    if k == 4:
        A = gaussian_bumps((512, 512, 256), 50, seed, np.float32)
        return Workload("c4_512x512x256_bumps_f32", A, (30, 30, 15), 10, 1,
                        "thosvd", "uniform", (8000, 8000, 8000), seed)
    raise ValueError(f"no config {k}")


CONFIGS = (1, 2, 3, 4)


def serving_shape(req_id: int, base_seed: int = 1000):
    """(dims, ranks) of a serving request without generating its tensor."""
    rng = np.random.default_rng(base_seed + req_id)
    dims = tuple(int(x) for x in rng.integers(32, 385, size=3))
    while True:
        ranks = tuple(int(x) for x in rng.integers(4, 25, size=3))
        ok = all(ranks[n] <= dims[n] and
                 ranks[n] <= int(np.prod([ranks[m] for m in range(3) if m != n]))
                 for n in range(3))
        if ok:
            break
    return dims, ranks


def serving_request(req_id: int, base_seed: int = 1000, dtype=np.float32):
    """One request of the serving stream: modes U{32..384}, ranks U{4..24}.

    Ranks are redrawn until mu_n <= I_n and mu_n <= prod_{m != n} mu_m (a
    feasible multilinear rank).  Gaussian core, orthonormal factors, noise 1e-3.
    Returns (A, ranks, samples) with samples T_n = 4*mu_n.
    """
    dims, ranks = serving_shape(req_id, base_seed)
    A = low_rank_plus_noise(dims, ranks, 1e-3, base_seed + req_id, dtype)
    return A, ranks, tuple(4 * r for r in ranks)


def serving_request_device(req_id: int, base_seed: int = 1000, device="cuda"):
    """A serving request generated in device memory (for long request streams).

    Same shape, ranks, core and factors as ``serving_request`` (numpy draws);
    the signal is assembled in float64 on the device and the noise is drawn
    with torch's generator on the device seeded with base_seed + req_id, so the
    tensor is a different sample of the same distribution.  Returns
    (X, ranks, samples) with X a column-major float32 device tensor.
    """
    import torch
    dims, ranks = serving_shape(req_id, base_seed)
    rng = np.random.default_rng(base_seed + req_id)
    C = rng.standard_normal(tuple(ranks)[::-1]).T
    U = [orth(rng.standard_normal((dims[n], ranks[n]))) for n in range(3)]
    f64 = dict(dtype=torch.float64, device=device)
    # B[i,j,k] = sum_abc C[a,b,c] U1[i,a] U2[j,b] U3[k,c], built as the
    # C-ordered array of reversed shape (k, j, i) so that its transpose is
    # the Fortran-ordered tensor.
    Ct = torch.as_tensor(np.ascontiguousarray(C.T), **f64)          # (c, b, a)
    U1, U2, U3 = (torch.as_tensor(u, **f64) for u in U)
    T = torch.matmul(Ct.reshape(-1, ranks[0]), U1.t().contiguous())  # (c*b, i)
    T = T.reshape(ranks[2], ranks[1], dims[0]).permute(0, 2, 1).reshape(-1, ranks[1])
    T = torch.matmul(T, U2.t().contiguous())                         # (c*i, j)
    T = T.reshape(ranks[2], dims[0], dims[1]).permute(1, 2, 0).reshape(-1, ranks[2])
    T = torch.matmul(T, U3.t().contiguous())                         # (i*j, k)
    B = T.reshape(dims[0], dims[1], dims[2]).permute(2, 1, 0).contiguous()  # (k, j, i)
    g = torch.Generator(device=device)
    g.manual_seed(base_seed + req_id)
    E = torch.randn(B.shape, generator=g, **f64)
    scale = 1e-3 * float(torch.linalg.vector_norm(B)) / math.sqrt(B.numel())
    X = (B + scale * E).to(torch.float32)
    return X.permute(2, 1, 0), ranks, tuple(4 * r for r in ranks)


def _colmajor(T):
    """A C-contiguous torch tensor rearranged in memory to column-major order
    (same logical shape and values)."""
    order = tuple(range(T.dim() - 1, -1, -1))
    return T.permute(order).contiguous().permute(order)


def _device_signal(core, factors, device):
    """B = core x_1 U_1 ... x_N U_N in float64 on the device (C-contiguous)."""
    import torch
    f64 = dict(dtype=torch.float64, device=device)
    B = torch.as_tensor(np.ascontiguousarray(core), **f64)
    for n, U in enumerate(factors):
        Ut = torch.as_tensor(np.ascontiguousarray(U), **f64)
        B = torch.movedim(torch.tensordot(Ut, B.contiguous(), dims=([1], [n])), 0, n)
    return B.contiguous()


def _device_noise(B, gamma, seed, dtype, device):
    import torch
    if gamma == 0.0:
        return _colmajor(B.to(dtype))
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    scale = gamma * float(torch.linalg.vector_norm(B)) / math.sqrt(B.numel())
    E = torch.randn(B.shape, generator=g, dtype=torch.float64, device=device)
    return _colmajor((B + scale * E).to(dtype))


def tucker_noise_device(dims, core_dims, gamma, seed, core="uniform", device="cuda",
                        dtype=None):
    """Eq. (9) tensor assembled on the device: A = B + gamma ||B||_F /
    sqrt(prod I_n) E, B = C x_1 A_1 ... x_N A_N with C iid U(0,1)
    (core="uniform", the paper's choice) or N(0,1) (core="gauss"), A_n an
    orthonormal basis of a standard Gaussian I_n x r_n matrix.  The core and
    factors are numpy draws (same order as ``low_rank_plus_noise``); the noise
    is drawn on the device with torch's generator seeded with ``seed``.
    Returns a column-major float32 (or ``dtype``) device tensor."""
    import torch
    rng = np.random.default_rng(seed)
    N = len(dims)
    if core == "uniform":
        C = rng.random(tuple(core_dims)[::-1]).T
    elif core == "gauss":
        C = rng.standard_normal(tuple(core_dims)[::-1]).T
    else:
        raise ValueError(core)
    U = [orth(rng.standard_normal((dims[n], core_dims[n]))) for n in range(N)]
    B = _device_signal(C, U, device)
    return _device_noise(B, gamma, seed, dtype or torch.float32, device)


def tendiag_noise_device(dims, decay, gamma, seed, device="cuda", dtype=None):
    """Section 6.3 tensor on the device: B = tendiag(v) x_1 A_1 ... x_N A_N
    (r = len(v) terms sum_i v_i a_i^(1) o ... o a_i^(N), A_n orthonormal
    I_n x r), plus relative noise gamma as in Eq. (9)."""
    import torch
    rng = np.random.default_rng(seed)
    N = len(dims)
    r = len(decay)
    U = [orth(rng.standard_normal((dims[n], r))) for n in range(N)]
    f64 = dict(dtype=torch.float64, device=device)
    v = torch.as_tensor(np.asarray(decay, dtype=np.float64), **f64)
    # B_(1) = A_1 diag(v) (A_N kr ... kr A_2)^T, built as C-ordered (I_1, ..., I_N)
    K = torch.as_tensor(np.ascontiguousarray(U[N - 1]), **f64)        # (I_N, r)
    for n in range(N - 2, 0, -1):
        Un = torch.as_tensor(np.ascontiguousarray(U[n]), **f64)      # (I_n, r)
        K = (Un[:, None, :] * K[None, :, :]).reshape(-1, r)           # (I_n * ..., r)
    A1 = torch.as_tensor(np.ascontiguousarray(U[0]), **f64) * v[None, :]
    B = torch.matmul(A1, K.t().contiguous()).reshape(tuple(dims))
    return _device_noise(B, gamma, seed, dtype or torch.float32, device)


def eq9_samples(alpha, dims, ranks, sthosvd):
    """T_n = ceil(alpha prod_{m != n} I_m) for Alg. 4 and ceil(alpha mu_1 ...
    mu_{n-1} I_{n+1} ... I_N) for Alg. 5 (the setting of Section 4.3)."""
    N = len(dims)
    out = []
    for n in range(N):
        p = 1
        for m in range(N):
            if m == n:
                continue
            p *= (ranks[m] if (sthosvd and m < n) else dims[m])
        out.append(int(math.ceil(alpha * p)))
    return tuple(out)


def sparse_cp_device(dims, n_terms, density, gamma, seed, device="cuda", dtype=None):
    """Sparse tensor of Sections 6.1 / 6.5: sum_i c_i x_i o y_i o z_i (o ...)
    with c_i = gamma / i^2 for i <= 50 and 1 / i^2 after, every factor vector
    sparse -- ceil(density I_n) nonzero entries at distinct uniformly drawn
    positions, N(0,1) values (the paper fixes only the density).  Built on the
    device in float64, returned column-major in float32 (or ``dtype``)."""
    import torch
    rng = np.random.default_rng(seed)
    N = len(dims)
    c = np.array([(gamma if i <= 50 else 1.0) / float(i) ** 2 for i in range(1, n_terms + 1)])
    U = []
    for n in range(N):
        F = np.zeros((dims[n], n_terms))
        k = int(math.ceil(density * dims[n]))
        for i in range(n_terms):
            pos = rng.choice(dims[n], size=k, replace=False)
            F[pos, i] = rng.standard_normal(k)
        U.append(F)
    f64 = dict(dtype=torch.float64, device=device)
    K = torch.as_tensor(np.ascontiguousarray(U[N - 1]), **f64)
    for n in range(N - 2, 0, -1):
        Un = torch.as_tensor(np.ascontiguousarray(U[n]), **f64)
        K = (Un[:, None, :] * K[None, :, :]).reshape(-1, n_terms)
    A1 = torch.as_tensor(np.ascontiguousarray(U[0]), **f64) * torch.as_tensor(c, **f64)[None, :]
    B = torch.matmul(A1, K.t().contiguous()).reshape(tuple(dims))
    return _colmajor(B.to(dtype or torch.float32))


def csc_mode1(X):
    """Compressed sparse columns of the mode-1 unfolding of a column-major
    tensor X (torch, any device): (colptr int64 [J_1 + 1], rowidx int32
    [nnz], vals [nnz]), rows increasing within each column."""
    import torch
    I1 = X.shape[0]
    J1 = X.numel() // I1
    order = tuple(range(X.dim() - 1, -1, -1))
    M = X.permute(order).reshape(J1, I1)      # row j = column j of A_(1)
    nz = torch.nonzero(M)                     # (j, i) in row-major order
    vals = M[nz[:, 0], nz[:, 1]].contiguous()
    counts = torch.bincount(nz[:, 0], minlength=J1)
    colptr = torch.zeros(J1 + 1, dtype=torch.int64, device=X.device)
    colptr[1:] = torch.cumsum(counts, 0)
    return colptr, nz[:, 1].to(torch.int32).contiguous(), vals
