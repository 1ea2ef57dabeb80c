"""Host-only checks of the C ABI (no device work): the library loads, exports
every function include/tucker_rand.h declares, and validates arguments the
way the header documents (workspace sizing runs the same validation as the
drivers, without launching anything)."""
import ctypes

import pytest
import torch

import paper_2303_11612_amd as tr
from paper_2303_11612_amd import _abi


def test_library_exports_every_header_symbol():
    L = _abi.lib()
    syms = _abi.header_symbols()
    assert "tucker_rand_thosvd" in syms and "tucker_rand_sthosvd" in syms
    assert "tucker_rand_sample" in syms and "tucker_rand_workspace_size" in syms
    missing = [s for s in syms if not hasattr(L, s)]
    assert missing == []
    assert set(_abi._SIGS) == set(syms)


def test_status_strings():
    assert tr.tucker_rand_status_string(0) == "ok"
    assert "invalid" in tr.tucker_rand_status_string(1)
    assert "workspace" in tr.tucker_rand_status_string(2)
    assert tr.tucker_rand_status_string(99) == "unknown status"


def _ws(*a, **k):
    return tr.tucker_rand_workspace_size(*a, **k)


def test_workspace_sizes_grow_with_problem():
    a = _ws((64, 64, 64), (5, 5, 5), 5, 1, dtype=torch.float64, sthosvd=False)
    b = _ws((128, 64, 64), (5, 5, 5), 5, 1, dtype=torch.float64, sthosvd=False)
    assert 0 < a < b
    c = _ws((400, 400, 400), (10, 10, 10), 10, 1, "nearly_optimal", (4000,) * 3)
    # norms, weights and prefix sums of 160000 columns plus two shrunk tensors
    assert c >= 3 * 8 * 160000 + 2 * 8 * 10 * 400 * 400


@pytest.mark.parametrize("bad", [
    dict(dims=(4, 4, 4), ranks=(5, 2, 2)),            # mu > I
    dict(dims=(4, 4, 4), ranks=(0, 2, 2)),            # mu < 1
    dict(dims=(4, 4, 4), ranks=(2, 2)),               # wrong length
    dict(dims=(4, 4, 4), ranks=(2, 2, 2), power=0),   # q < 1
    dict(dims=(4, 4, 4), ranks=(2, 2, 2), oversample=-1),
    dict(dims=(4, 4, 4), ranks=(2, 2, 2), prob="uniform", samples=(0, 1, 1)),
    dict(dims=(0, 4, 4), ranks=(1, 2, 2)),
])
def test_invalid_arguments_rejected(bad):
    kw = dict(oversample=2, power=1, prob="none", samples=None)
    kw.update({k: v for k, v in bad.items() if k not in ("dims", "ranks")})
    with pytest.raises((_abi.TuckerRandError, ValueError)) as e:
        _ws(bad["dims"], bad["ranks"], **kw)
    if isinstance(e.value, _abi.TuckerRandError):
        assert e.value.code == _abi.TR_EINVAL


def test_sthosvd_rank_checked_against_shrunk_unfolding():
    # mode 3 of the shrunk 1 x 1 x 9 tensor has J_3 = 1 < mu_3 = 2
    _ws((6, 6, 9), (1, 1, 1), 2, 1)
    with pytest.raises(_abi.TuckerRandError):
        _ws((6, 6, 9), (1, 1, 2), 2, 1, sthosvd=True)
    _ws((6, 6, 9), (1, 1, 2), 2, 1, sthosvd=False)   # T-HOSVD: J_3 = 36


def test_unsupported_requests():
    with pytest.raises(_abi.TuckerRandError) as e:
        _ws((200, 200, 200), (130, 10, 10), 10, 1)       # s = 140 > 128
    assert e.value.code == _abi.TR_ENOTSUP
    # 64 < s <= 128: the plain power scheme only
    assert _ws((200, 200, 200), (100, 10, 10), 10, 1) > _ws((200, 200, 200), (50, 10, 10), 10, 1)
    for flags in (["stabilized_power"], ["related_form"]):
        with pytest.raises(_abi.TuckerRandError) as e:
            tr.tucker_rand_workspace_size((200, 200, 200), (100, 10, 10), 10, 2, "none",
                                          flags=flags)
        assert e.value.code == _abi.TR_ENOTSUP
    # low-precision power products: I_n <= 512 and s_n <= 48
    with pytest.raises(_abi.TuckerRandError) as e:
        _ws((600, 20, 20), (4, 4, 4), 4, 1, precision="bf16")
    assert e.value.code == _abi.TR_ENOTSUP
    with pytest.raises(_abi.TuckerRandError) as e:
        _ws((100, 100, 100), (40, 4, 4), 10, 1, precision="fp8e4m3")   # s = 50
    assert e.value.code == _abi.TR_ENOTSUP
    assert _ws((20, 20, 20), (4, 4, 4), 4, 1, precision="bf16") > 0
    with pytest.raises(_abi.TuckerRandError) as e:
        _ws((20, 20, 20), (4, 4, 4), 4, 1, precision=7)
    assert e.value.code == _abi.TR_EINVAL


def test_null_pointers_rejected_before_launch():
    L = _abi.lib()
    assert L.tucker_rand_workspace_size(None, 0, 0, None) == _abi.TR_EINVAL
    assert L.tucker_rand_gaussian(4, 2, 0, 0, None, None) == _abi.TR_EINVAL
    assert L.tucker_rand_factor(None, 4, 2, 1, None, None, None, 0, None) == _abi.TR_EINVAL
    assert L.tucker_rand_sample(None, 10, 5, 1, 0, 0, None, None, None, 0, None, None) == \
        _abi.TR_EINVAL
    p, keep = tr._params((8, 8), (2, 2), 2, 1, "none", None, 0, "native")
    q = (ctypes.c_void_p * 2)(None, None)
    rc = L.tucker_rand_thosvd(ctypes.byref(p), 0, None, q, None, None, 0, None, None)
    assert rc == _abi.TR_EINVAL
    assert L.tucker_rand_timer_read(None, 0, None, None, None, None) == _abi.TR_EINVAL


def test_binding_refuses_host_tensors():
    A = torch.zeros(4, 4, 4, dtype=torch.float64)
    with pytest.raises(ValueError):
        tr.tucker_rand_thosvd(A, (2, 2, 2), 1, 1)


def test_noalloc_scratch_size_matches_header():
    import re
    with open(_abi.HEADER) as f:
        m = re.search(r"#define\s+TR_NOALLOC_SCRATCH_BYTES\s+\(\(size_t\)(\d+)\s*<<\s*(\d+)\)",
                      f.read())
    assert m, "TR_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == _abi.NOALLOC_SCRATCH_BYTES
    # the headline 400^3 sampled ST-HOSVD fits the fixed scratch
    import torch
    import paper_2303_11612_amd as tr
    need = tr.tucker_rand_workspace_size((400, 400, 400), (10, 10, 10), 10, 1,
                                         "nearly_optimal", (4000, 4000, 4000), 0, torch.float32)
    assert need <= _abi.NOALLOC_SCRATCH_BYTES


def test_flag_bits_validated_on_host():
    import paper_2303_11612_amd as tr
    base = tr.tucker_rand_workspace_size((40, 30, 20), (4, 4, 4), 4, 2, "none")
    stab = tr.tucker_rand_workspace_size((40, 30, 20), (4, 4, 4), 4, 2, "none",
                                         flags=["stabilized_power"])
    assert stab > base   # per mode: the orthonormal iterate, Rbar, U'
    assert tr.tucker_rand_workspace_size((40, 30, 20), (4, 4, 4), 4, 2, "none",
                                         flags=["unfused_power"]) == base
    assert tr.tucker_rand_workspace_size((40, 30, 20), (4, 4, 4), 4, 2, "none",
                                         flags=["related_form"]) > base
    for bad in (0x8, 0x10, 0x80000000):
        with pytest.raises(_abi.TuckerRandError, match="invalid argument"):
            tr.tucker_rand_workspace_size((40, 30, 20), (4, 4, 4), 4, 2, "none", flags=bad)


def test_adaptive_arguments_validated_on_host():
    # tol <= 0, relative outside {0, 1} or missing outputs: TR_EINVAL before
    # anything is launched (no device pointer is touched)
    p, _keep = tr._params((20, 16, 12), (4, 4, 4), 4, 1, "none", None, 0, "native")
    ranks = (ctypes.c_int64 * 3)()
    bound = ctypes.c_double()
    qp = (ctypes.c_void_p * 3)(1, 1, 1)
    for tol, rel in ((0.0, 1), (-1.0, 0), (0.1, 2)):
        rc = _abi.lib().tucker_rand_adaptive(ctypes.byref(p), 0, 1, tol, rel, ctypes.c_void_p(1),
                                             qp, ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 30,
                                             ranks, ctypes.byref(bound), None, None)
        assert rc == _abi.TR_EINVAL


def _breq(ranks, samples, prob="nearly_optimal", oversample=4, power=1, seed=0):
    return tr.BatchRequest(None, ranks, samples, oversample, power, prob, seed)


def test_batch_workspace_and_limits_on_host():
    a = _breq((4, 4, 3), (300, 200, 100))
    b = _breq((6, 5, 5), (900, 400, 50), prob="uniform", seed=3)
    one = tr.tucker_rand_batch_workspace_size([a], dims=[(40, 30, 20)])
    two = tr.tucker_rand_batch_workspace_size([a, b], dims=[(40, 30, 20), (64, 48, 32)])
    assert 0 < one < two
    # T_n > J_n is accepted (the exact product for that mode)
    assert tr.tucker_rand_batch_workspace_size([_breq((4, 4, 3), (5000, 5000, 5000))],
                                               dims=[(40, 30, 20)]) > 0

    def code(reqs, dims, dtype=torch.float32):
        with pytest.raises(_abi.TuckerRandError) as e:
            tr.tucker_rand_batch_workspace_size(reqs, dtype, dims)
        return e.value.code

    # mixed orders, prob none, a bad rank: invalid or unsupported, before any launch
    assert code([a, _breq((2, 2), (10, 10))], [(40, 30, 20), (8, 8)]) == _abi.TR_EINVAL
    assert code([_breq((4, 4, 3), (300, 200, 100), prob="none")], [(40, 30, 20)]) == \
        _abi.TR_ENOTSUP
    assert code([_breq((41, 4, 3), (300, 200, 100))], [(40, 30, 20)]) == _abi.TR_EINVAL
    # the grouped kernels' limits: I_n <= 512, s_n <= 48, min(T_n, J_n) <= 8192
    assert code([_breq((4, 4, 3), (300, 200, 100))], [(600, 20, 20)]) == _abi.TR_ENOTSUP
    assert code([_breq((40, 4, 3), (300, 200, 100), oversample=10)], [(100, 60, 50)]) == \
        _abi.TR_ENOTSUP
    assert code([_breq((4, 4, 3), (9000, 200, 100))], [(100, 100, 100)]) == _abi.TR_ENOTSUP
    L = _abi.lib()
    out = ctypes.c_size_t()
    assert L.tucker_rand_batch_workspace_size(0, None, 0, ctypes.byref(out)) == _abi.TR_EINVAL
    arr, _keep = tr._batch_params([a], [(40, 30, 20)])
    assert L.tucker_rand_batch_workspace_size(1, arr, 5, ctypes.byref(out)) == _abi.TR_EINVAL
    # null tensors are rejected before anything is copied or launched
    nul = (ctypes.c_void_p * 1)(None)
    qn = (ctypes.POINTER(ctypes.c_void_p) * 1)(None)
    assert L.tucker_rand_sthosvd_batch(1, arr, 1, nul, qn, nul, None, 0, None, None) == \
        _abi.TR_EINVAL


def test_sparse_entry_validated_on_host():
    L = _abi.lib()
    p, _keep = tr._params((20, 16, 12), (4, 4, 4), 4, 1, "nearly_optimal", (50, 40, 30), 0,
                          "native")
    q = (ctypes.c_void_p * 3)(1, 1, 1)
    one = ctypes.c_void_p(1)
    # missing colptr / negative nnz / missing values with nnz > 0
    assert L.tucker_rand_sthosvd_csc(ctypes.byref(p), 0, 10, None, one, one, q, one, one,
                                     1 << 30, None, None) == _abi.TR_EINVAL
    assert L.tucker_rand_sthosvd_csc(ctypes.byref(p), 0, -1, one, one, one, q, one, one,
                                     1 << 30, None, None) == _abi.TR_EINVAL
    assert L.tucker_rand_sthosvd_csc(ctypes.byref(p), 0, 10, one, None, one, q, one, one,
                                     1 << 30, None, None) == _abi.TR_EINVAL
    # the first mode must be sampled (exact products on the sparse tensor are not built)
    for prob, samples in (("none", None), ("nearly_optimal", (500, 40, 30))):
        p2, _k2 = tr._params((20, 16, 12), (4, 4, 4), 4, 1, prob, samples, 0, "native")
        assert L.tucker_rand_sthosvd_csc(ctypes.byref(p2), 0, 10, one, one, one, q, one, one,
                                         1 << 30, None, None) == _abi.TR_ENOTSUP
    p3, _k3 = tr._params((20, 16, 12), (4, 4, 4), 4, 1, "nearly_optimal", (50, 40, 30), 0,
                         "bf16")
    assert L.tucker_rand_sthosvd_csc(ctypes.byref(p3), 0, 10, one, one, one, q, one, one,
                                     1 << 30, None, None) == _abi.TR_ENOTSUP
