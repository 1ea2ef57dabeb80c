"""The allocation-free ST-HOSVD entry point (tucker_rand_sthosvd_noalloc),
called through the C ABI, against tucker_rand_sthosvd on the same inputs.

Both run the same kernels; only the workspace differs (the library's fixed
device scratch instead of a caller buffer), so factors and core are expected
to agree bit for bit.  The bar asserted is the FP64 parity bar of 1e-10
relative (FP32 outputs: 1e-6, their rounding), plus identical sampled
indices.  Two calls in a row, the second with a smaller input, check that the
scratch left by one call does not leak into the next.
"""
import ctypes
from ctypes import byref, c_void_p

import numpy as np
import pytest
import torch

import synth
import paper_2303_11612_amd as tr
from paper_2303_11612_amd import _abi

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = torch.linalg.norm(b.double())
    return float(torch.linalg.norm(a.double() - b.double()) / (nb if nb > 0 else 1.0))


def _both(A, ranks, K, q, prob, samples, seed):
    X = tr.to_device(A)
    Qa, ca, ia = tr.tucker_rand_sthosvd(X, ranks, K, q, prob, samples, seed, diag=True)
    Qb, cb, ib = tr.tucker_rand_sthosvd_noalloc(X, ranks, K, q, prob, samples, seed,
                                                diag=True)
    torch.cuda.synchronize()
    return (Qa, ca, ia), (Qb, cb, ib)


def _check(ref, got, tol):
    (Qa, ca, ia), (Qb, cb, ib) = ref, got
    assert int(ib["status"].item()) == 0
    for n in range(len(Qa)):
        assert _rel(Qb[n], Qa[n]) <= tol, n
        assert torch.equal(ib["sigma"][n], ia["sigma"][n]), n
        if "indices" in ia:
            assert torch.equal(ib["indices"][n], ia["indices"][n]), n
    assert _rel(cb, ca) <= tol


def test_noalloc_matches_sthosvd_twice_shrinking():
    # first call: a sampled float32 problem near the scratch's intended size
    A1 = synth.low_rank_plus_noise((300, 280, 260), (10, 10, 10), 1e-4, 11, np.float32)
    args1 = ((10, 10, 10), 10, 1, "nearly_optimal", (3000, 3000, 3000), 5)
    ref1, got1 = _both(A1, *args1)
    _check(ref1, got1, 1e-6)
    # second call, smaller and exact, float64, q = 2: nothing of the first
    # call's scratch contents may reach it
    A2 = synth.low_rank_plus_noise((41, 37, 29), (5, 4, 4), 1e-3, 12, np.float64)
    args2 = ((4, 4, 3), 5, 2, "none", None, 9)
    ref2, got2 = _both(A2, *args2)
    _check(ref2, got2, 1e-10)
    # the same call again gives the same bits
    X2 = tr.to_device(A2)
    Qc, cc, _ = tr.tucker_rand_sthosvd_noalloc(X2, *args2)
    torch.cuda.synchronize()
    assert torch.equal(cc, got2[1])
    assert all(torch.equal(Qc[n], got2[0][n]) for n in range(3))


def test_noalloc_rejects_oversized_workspace():
    # 100^4 float32 exact with rank 20 needs ~709 MiB of workspace: rejected on
    # the host before anything runs (TR_ENOMEM), for any input pointer
    dims, ranks = (100, 100, 100, 100), (20, 20, 20, 20)
    need = tr.tucker_rand_workspace_size(dims, ranks, 10, 2, "none", None, 0, torch.float32)
    assert need > _abi.NOALLOC_SCRATCH_BYTES
    p, _keep = tr._params(dims, ranks, 10, 2, "none", None, 0, "native")
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    qptrs = (c_void_p * 4)(*([dummy.data_ptr()] * 4))
    rc = _abi.lib().tucker_rand_sthosvd_noalloc(
        byref(p), _abi.TR_F32, c_void_p(dummy.data_ptr()), qptrs, c_void_p(dummy.data_ptr()),
        None, c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _abi.TR_ENOMEM
    assert torch.count_nonzero(dummy).item() == 0


def test_noalloc_on_side_stream_with_preallocated_outputs():
    A = synth.low_rank_plus_noise((64, 48, 40), (6, 5, 4), 1e-3, 13, np.float64)
    X = tr.to_device(A)
    ranks = (5, 4, 4)
    Qa, ca, _ = tr.tucker_rand_sthosvd(X, ranks, 4, 1, "uniform", (500, 200, 100), 3)
    torch.cuda.synchronize()
    out = ([tr.colmajor_empty((A.shape[n], ranks[n]), torch.float64) for n in range(3)],
           tr.colmajor_empty(ranks, torch.float64))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    Qb, cb, _ = tr.tucker_rand_sthosvd_noalloc(X, ranks, 4, 1, "uniform", (500, 200, 100), 3,
                                               stream=s, out=out)
    s.synchronize()
    assert torch.equal(cb, ca)
    assert all(torch.equal(Qb[n], Qa[n]) for n in range(3))
