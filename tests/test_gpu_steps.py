"""GPU parity of each step of the range finder against the FP64 oracle, called
through the C ABI.  Shapes span several workgroup tiles plus a ragged tail,
and every 3-D view kind (L == 1 and L > 1).

Bars: integer results (sampled indices) and the column norms and rescales
computed from identical inputs are bit-exact; float64 products within 1e-12
relative (they differ from numpy only in summation order); the Gaussian within
1e-13 absolute (the device's log/cos/sin are not the host's libm).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2303_11612_amd as tr
from paper_2303_11612_amd import _abi

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _np(t):
    return t.detach().cpu().numpy()


def _rand_tensor(shape, dtype, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal(shape[::-1]).T * np.linspace(0.5, 2.0, shape[-1])
    return np.asfortranarray(A.astype(dtype))


def _views(shape):
    N = len(shape)
    out = []
    for n in range(N):
        L = int(np.prod(shape[:n]))
        R = int(np.prod(shape[n + 1:]))
        out.append((n, L, shape[n], R))
    return out


@pytest.mark.parametrize("I,s,mode,seed", [(64, 10, 0, 0), (400, 20, 2, 7), (37, 3, 1, 2**63 + 5),
                                           (1, 1, 0, 1), (513, 33, 4, 99)])
def test_gaussian_matches_oracle(I, s, mode, seed):
    G = _np(tr.tucker_rand_gaussian(I, s, mode, seed))
    Go = oracle.gaussian_matrix(I, s, mode, seed)
    assert G.shape == Go.shape
    assert np.max(np.abs(G - Go)) < 1e-13


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(300, 70, 3), (37, 23, 11), (5, 600, 2), (1000, 1, 1),
                                   (4, 50, 3), (8, 33, 5), (400, 20, 20)])
def test_colnorms_bit_exact(dtype, shape):
    A = _rand_tensor(shape, dtype, 3)
    X = tr.to_device(A)
    for n, L, I, R in _views(shape):
        norms, mb = tr.tucker_rand_colnorms(X, L, I, R)
        want = oracle.column_sq_norms(oracle.unfold(A.astype(np.float64), n))
        got = _np(norms)
        assert np.array_equal(got, want), (shape, n)
        assert _np(mb)[0] == want.max().view(np.int64)


def _norm_vectors():
    rng = np.random.default_rng(11)
    J = 160000
    yield "c2_shape", J, rng.random(J) ** 6 * 3.0
    n = rng.random(5000)
    n[::7] = 0.0
    n[3] = 1e-300
    yield "zeros", 5000, n
    yield "tiny", 3, np.array([1.0, 2.0, 0.5])
    yield "one", 1, np.array([4.0])
    # the largest mode sampled in one launch (every workgroup scans the
    # weights in LDS) and the smallest one sampled by the three launches
    for J in (6144, 6145):
        n = rng.random(J) ** 3
        n[::5] = 0.0
        yield f"one_launch_edge_{J}", J, n
    # more than 1024 scan blocks of 1024 columns: the block offsets are
    # scanned by their own launch instead of inside the prefix-sum kernel
    J = 1200000
    yield "many_blocks", J, rng.random(J) ** 4


@pytest.mark.parametrize("case", list(_norm_vectors()), ids=lambda c: c[0])
@pytest.mark.parametrize("T", [1, 7, 4000])
def test_sampler_bit_exact(case, T):
    _, J, n = case
    for mode, seed in ((0, 0), (2, 12345)):
        idx, scale, status = tr.tucker_rand_sample(torch.tensor(n, device=DEV), J, T,
                                                   "nearly_optimal", seed, mode)
        xi, sc, w, W = oracle.randsample(n, J, T, oracle.PROB_NEARLY_OPTIMAL, seed, mode)
        assert np.array_equal(_np(idx), xi)
        assert np.array_equal(_np(scale), sc)       # bitwise: same IEEE operations
        assert _np(status)[0] == 0


@pytest.mark.parametrize("J,T", [(160000, 4000), (131072, 8000), (5, 50), (1, 3)])
def test_uniform_sampler_bit_exact(J, T):
    idx, scale, _ = tr.tucker_rand_sample(None, J, T, "uniform", 9, 1)
    xi, sc, _, _ = oracle.randsample(None, J, T, oracle.PROB_UNIFORM, 9, 1)
    assert np.array_equal(_np(idx), xi)
    assert np.array_equal(_np(scale), sc)


def test_sampler_flags_all_zero_distribution():
    idx, scale, status = tr.tucker_rand_sample(torch.zeros(100, dtype=torch.float64,
                                                           device=DEV), 100, 10,
                                               "nearly_optimal", 0, 0)
    assert _np(status)[0] & _abi.TR_DEV_ZERO_DIST
    assert np.all(_np(scale) == 0.0)
    n = np.ones(10)
    n[4] = np.nan
    _, _, status = tr.tucker_rand_sample(torch.tensor(n, device=DEV), 10, 10,
                                         "nearly_optimal", 0, 0)
    assert _np(status)[0] & _abi.TR_DEV_NONFINITE


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_gather_bit_exact(dtype):
    shape = (45, 31, 17)
    A = _rand_tensor(shape, dtype, 5)
    X = tr.to_device(A)
    rng = np.random.default_rng(0)
    for n, L, I, R in _views(shape):
        idx = rng.integers(0, L * R, size=333)
        idx[:3] = [0, L * R - 1, 0]
        Cp = _np(tr.tucker_rand_gather(X, L, I, R, torch.tensor(idx, device=DEV)))
        want = oracle.unfold(A, n)[:, idx]
        assert Cp.dtype == A.dtype and np.array_equal(Cp, want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(12, 40, 100), (7, 300, 70)])
def test_gather_many_slabs_bit_exact(dtype, shape):
    """Inner-mode views with many slabs (R >= 64): uniform samples with
    repeats, every sample in one slab, and 8192 / 8193 samples."""
    A = _rand_tensor(shape, dtype, 6)
    X = tr.to_device(A)
    rng = np.random.default_rng(1)
    L, I, R = shape[0], shape[1], shape[2]
    want_all = oracle.unfold(A, 1)
    cases = [rng.integers(0, L * R, size=333),
             5 * L + rng.integers(0, L, size=500),
             rng.integers(0, L * R, size=8192),
             rng.integers(0, L * R, size=8193)]
    for idx in cases:
        idx[:2] = [0, L * R - 1]
        Cp = _np(tr.tucker_rand_gather(X, L, I, R, torch.tensor(idx, device=DEV)))
        assert Cp.dtype == A.dtype and np.array_equal(Cp, want_all[:, idx]), (shape, len(idx))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("q", [1, 2])
def test_power_products_match_oracle(dtype, q):
    shape = (70, 90, 33)
    A = _rand_tensor(shape, dtype, 8)
    X = tr.to_device(A)
    for n, L, I, R in _views(shape):
        s = 12
        G = oracle.gaussian_matrix(I, s, n, 4)
        M = oracle.unfold(A.astype(np.float64), n)
        C = _np(tr.tucker_rand_power(X, L, I, R, tr.to_device(G), q))
        want = oracle.power_sketch(M, G, q)
        assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want), n
    # column-weighted form (C' D C'^T)^q G used by the sampled products
    I, T = 70, 500
    Cp = _rand_tensor((I, T), dtype, 9)
    d = np.random.default_rng(1).random(T) + 0.5
    G = oracle.gaussian_matrix(I, 8, 0, 1)
    C = _np(tr.tucker_rand_power(tr.to_device(Cp), 1, I, T, tr.to_device(G), q,
                                 torch.tensor(d, device=DEV)))
    Ms = Cp.astype(np.float64) * np.sqrt(d)[None, :]
    want = oracle.power_sketch(Ms, G, q)
    assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("s", [16, 17, 32])
def test_power_products_wide_sketch(dtype, s):
    """Sketch widths past one 16-column group, rows up to 128 (eight row
    chunks) and a ragged last column tile, plain and column-weighted."""
    shape = (128, 45, 21)
    A = _rand_tensor(shape, dtype, 11)
    X = tr.to_device(A)
    for n, L, I, R in _views(shape):
        if s > I:
            continue
        G = oracle.gaussian_matrix(I, s, n, 6)
        M = oracle.unfold(A.astype(np.float64), n)
        C = _np(tr.tucker_rand_power(X, L, I, R, tr.to_device(G), 1))
        want = oracle.power_sketch(M, G, 1)
        assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want), n
    I, T = 113, 1001
    Cp = _rand_tensor((I, T), dtype, 12)
    d = np.random.default_rng(2).random(T) + 0.5
    G = oracle.gaussian_matrix(I, s, 0, 3)
    C = _np(tr.tucker_rand_power(tr.to_device(Cp), 1, I, T, tr.to_device(G), 2,
                                 torch.tensor(d, device=DEV)))
    Ms = Cp.astype(np.float64) * np.sqrt(d)[None, :]
    want = oracle.power_sketch(Ms, G, 2)
    assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("s", [12, 20, 32])
def test_power_products_rows_past_128(dtype, s):
    """Rows past the one-sweep kernel's 128 (144 to 512, not multiples of 16),
    L = 1 and L > 1 views, a ragged last column tile, q = 1 and 2, plain and
    column-weighted: the two-product form at these widths."""
    for shape in ((144, 300, 7), (512, 21, 9), (129, 17, 40), (400, 33, 12), (257, 6, 11)):
        A = _rand_tensor(shape, dtype, 13)
        X = tr.to_device(A)
        for n, L, I, R in _views(shape):
            if I <= 128 or s > I:
                continue
            for q in (1, 2):
                G = oracle.gaussian_matrix(I, s, n, 7)
                M = oracle.unfold(A.astype(np.float64), n)
                C = _np(tr.tucker_rand_power(X, L, I, R, tr.to_device(G), q))
                want = oracle.power_sketch(M, G, q)
                assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want), (shape, n, q)
    I, T = 333, 1001
    Cp = _rand_tensor((I, T), dtype, 14)
    d = np.random.default_rng(3).random(T) + 0.5
    G = oracle.gaussian_matrix(I, s, 0, 5)
    C = _np(tr.tucker_rand_power(tr.to_device(Cp), 1, I, T, tr.to_device(G), 2,
                                 torch.tensor(d, device=DEV)))
    Ms = Cp.astype(np.float64) * np.sqrt(d)[None, :]
    want = oracle.power_sketch(Ms, G, 2)
    assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want)


def _graded(I, s, seed, decay=0.6):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((I, s)))[0]
    V = np.linalg.qr(rng.standard_normal((s, s)))[0]
    return np.asfortranarray(U @ np.diag(decay ** np.arange(s)) @ V.T)


@pytest.fixture(params=["reg", "lds"])
def factor_variant(request, monkeypatch):
    """Both factor kernels: the register-resident one (default for s <= 48,
    I <= 512) and the LDS-resident one (every shape when forced)."""
    monkeypatch.setenv("TUCKER_RAND_FACTOR", request.param)
    return request.param


@pytest.mark.parametrize("I,s,mu", [(64, 10, 5), (400, 20, 10), (512, 40, 30), (100, 30, 20),
                                    (513, 16, 9), (1000, 24, 12), (2000, 12, 4), (7, 7, 7),
                                    (1, 1, 1), (33, 1, 1), (96, 64, 40), (256, 16, 16),
                                    (300, 16, 8), (256, 32, 32), (512, 32, 16), (400, 30, 20),
                                    (257, 17, 16), (2, 2, 1), (40, 31, 3), (256, 24, 24),
                                    (130, 21, 17), (400, 24, 16), (512, 17, 3), (200, 36, 36),
                                    (200, 19, 16), (256, 20, 16), (400, 20, 10), (300, 18, 17),
                                    (300, 33, 20), (256, 40, 40)])
def test_factor_matches_svd(I, s, mu, factor_variant):
    C = _graded(I, s, I + s)
    Q, sig = tr.tucker_rand_factor(tr.to_device(C), mu)
    Q, sig = _np(Q), _np(sig)
    Qo, so = oracle.leading_left_singular_vectors(C, mu)
    assert np.allclose(sig, so, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(Q.T @ Q - np.eye(mu))) < 1e-13
    # column c of either side is determined to ~u * sigma_1 / gap_c; both
    # errors add.  For the well-separated cases this is far below 1e-10.
    for c in range(mu):
        gap = min(so[c - 1] - so[c] if c else np.inf,
                  so[c] - so[c + 1] if c + 1 < len(so) else so[c])
        bound = max(1e-10, 20 * 2.2e-16 * so[0] / gap)
        assert np.linalg.norm(Q[:, c] - Qo[:, c]) <= bound, (c, bound)


def test_factor_of_strongly_graded_sketch(factor_variant):
    # spectrum like C_n = (A A^T) G_n for the 400^3 tensor: 0.25^k, then a noise floor
    I, s, mu = 400, 20, 10
    rng = np.random.default_rng(3)
    U = np.linalg.qr(rng.standard_normal((I, s)))[0]
    V = np.linalg.qr(rng.standard_normal((s, s)))[0]
    sv = np.concatenate([0.25 ** np.arange(10), 1e-11 * (1 + rng.random(10))])
    C = np.asfortranarray(U @ np.diag(sv) @ V.T)
    Q, sig = tr.tucker_rand_factor(tr.to_device(C), mu)
    Qo, so = oracle.leading_left_singular_vectors(C, mu)
    Q = _np(Q)
    assert np.allclose(_np(sig)[:mu], so[:mu], rtol=1e-10)
    for c in range(mu):   # column c is determined to ~u * sigma_1 / gap_c
        gap = min(so[c - 1] - so[c] if c else np.inf, so[c] - so[c + 1])
        assert np.linalg.norm(Q[:, c] - Qo[:, c]) <= 1e-14 * so[0] / gap + 1e-13


@pytest.mark.parametrize("I,s,mu,rank", [(50, 10, 5, 3), (400, 20, 10, 0), (300, 24, 12, 7)])
def test_factor_of_rank_deficient_sketch(I, s, mu, rank, factor_variant):
    # sigma_rank.. are exactly zero: the trailing columns of Q_n are any
    # orthonormal completion, so only the leading ones and orthonormality are compared
    rng = np.random.default_rng(I + rank)
    C = np.asfortranarray(rng.standard_normal((I, rank)) @ rng.standard_normal((rank, s))
                          if rank else np.zeros((I, s)))
    Q, sig = tr.tucker_rand_factor(tr.to_device(C), mu)
    Q, sig = _np(Q), _np(sig)
    Qo, so = oracle.leading_left_singular_vectors(C, mu)
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(sig))
    assert np.max(np.abs(Q.T @ Q - np.eye(mu))) < 1e-13
    scale = so[0] if rank else 1.0
    assert np.allclose(sig[:rank], so[:rank], rtol=1e-12)
    assert np.all(np.abs(sig[rank:]) <= 1e-13 * scale)
    for c in range(min(rank, mu)):
        gap = min(so[c - 1] - so[c] if c else np.inf, so[c] - so[c + 1] if c + 1 < rank else so[c])
        assert np.linalg.norm(Q[:, c] - Qo[:, c]) <= max(1e-10, 20 * 2.2e-16 * so[0] / gap)


@pytest.mark.parametrize("in_dt", [np.float32, np.float64])
@pytest.mark.parametrize("out_dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("mu", [3, 10, 20, 40])
@pytest.mark.parametrize("shape", [(61, 45, 300), (64, 30, 77), (400, 21, 19), (36, 5, 7)])
def test_ttm_matches_mode_product(in_dt, out_dt, mu, shape):
    # leading extents that are (not) multiples of 4 take the vector-load (or
    # scalar) form of the mode-1 product; 400 rows span 12.5 row steps
    A = _rand_tensor(shape, in_dt, 4)
    X = tr.to_device(A)
    rng = np.random.default_rng(mu)
    for n, L, I, R in _views(shape):
        m = min(mu, I)
        Q = np.linalg.qr(rng.standard_normal((I, m)))[0]
        Y = _np(tr.tucker_rand_ttm(X, L, I, R, tr.to_device(Q), out_dtype=out_dt))
        want = oracle.mode_product(A.astype(np.float64), Q.T, n).ravel(order="F")
        tol = 1e-13 if out_dt == torch.float64 else 2e-7
        assert np.linalg.norm(Y - want) <= tol * np.linalg.norm(want), (n, m)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("s", [65, 100, 128])
def test_power_products_sketch_past_64(dtype, s):
    """Sketch widths above 64 (five to eight 16-column groups)."""
    shape = (200, 45, 150)
    A = _rand_tensor(shape, dtype, 15)
    X = tr.to_device(A)
    for n, L, I, R in _views(shape):
        if s > I:
            continue
        G = oracle.gaussian_matrix(I, s, n, 8)
        M = oracle.unfold(A.astype(np.float64), n)
        C = _np(tr.tucker_rand_power(X, L, I, R, tr.to_device(G), 1))
        want = oracle.power_sketch(M, G, 1)
        assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want), n
    I, T = 150, 1001
    Cp = _rand_tensor((I, T), dtype, 16)
    d = np.random.default_rng(4).random(T) + 0.5
    G = oracle.gaussian_matrix(I, s, 0, 9)
    C = _np(tr.tucker_rand_power(tr.to_device(Cp), 1, I, T, tr.to_device(G), 2,
                                 torch.tensor(d, device=DEV)))
    Ms = Cp.astype(np.float64) * np.sqrt(d)[None, :]
    want = oracle.power_sketch(Ms, G, 2)
    assert np.linalg.norm(C - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("I,s,mu", [(200, 65, 50), (600, 110, 100), (128, 128, 128),
                                    (300, 100, 60), (1000, 90, 90), (129, 72, 1)])
def test_factor_wide_sketch(I, s, mu):
    """Sketches of 65..128 columns (the kernel with its s x s matrices in
    global scratch, Jacobi on R1 with two rows per lane)."""
    C = _graded(I, s, I + s, decay=0.9)
    Q, sig = tr.tucker_rand_factor(tr.to_device(C), mu)
    Q, sig = _np(Q), _np(sig)
    Qo, so = oracle.leading_left_singular_vectors(C, mu)
    assert np.allclose(sig, so, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(Q.T @ Q - np.eye(mu))) < 1e-13
    for c in range(mu):
        gap = min(so[c - 1] - so[c] if c else np.inf,
                  so[c] - so[c + 1] if c + 1 < len(so) else so[c])
        bound = max(1e-10, 20 * 2.2e-16 * so[0] / gap)
        assert np.linalg.norm(Q[:, c] - Qo[:, c]) <= bound, (c, bound)


@pytest.mark.parametrize("in_dt", [np.float32, np.float64])
@pytest.mark.parametrize("mu", [65, 100, 128])
def test_ttm_rank_past_64(in_dt, mu):
    shape = (200, 140, 30)
    A = _rand_tensor(shape, in_dt, 5)
    X = tr.to_device(A)
    rng = np.random.default_rng(mu)
    for n, L, I, R in _views(shape):
        if mu > I:
            continue
        Q = np.linalg.qr(rng.standard_normal((I, mu)))[0]
        Y = _np(tr.tucker_rand_ttm(X, L, I, R, tr.to_device(Q), out_dtype=torch.float64))
        want = oracle.mode_product(A.astype(np.float64), Q.T, n).ravel(order="F")
        assert np.linalg.norm(Y - want) <= 1e-13 * np.linalg.norm(want), (n, mu)
