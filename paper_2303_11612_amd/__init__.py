"""Randomized T-HOSVD / ST-HOSVD with the power scheme and approximate matrix
multiplication (Che, Wei, Yan) on AMD MI355X (gfx950).

This module is a thin binding over the C ABI of ``include/tucker_rand.h``: it
checks tensor layouts, allocates outputs and workspaces through torch (device
memory and streams only) and passes raw pointers.  Every arithmetic step runs
in the library's HIP kernels; if the library is missing, every call raises.

Tensors are column-major: a tensor of shape (I_1, ..., I_N) must have strides
(1, I_1, I_1 I_2, ...).  ``colmajor_empty`` and ``to_device`` make such tensors.
"""
from __future__ import annotations

import ctypes
import math
from ctypes import byref, c_double, c_int64, c_size_t, c_void_p
from typing import Optional, Sequence

import torch

from . import _abi
from ._abi import KC, PREC, PROB, TR_F32, TR_F64, check, lib

__all__ = [
    "colmajor_empty", "to_device", "is_colmajor", "Timer",
    "tucker_rand_workspace_size", "tucker_rand_thosvd", "tucker_rand_sthosvd",
    "tucker_rand_sthosvd_noalloc", "tucker_rand_adaptive",
    "BatchRequest", "tucker_rand_batch_workspace_size", "tucker_rand_sthosvd_batch",
    "tucker_rand_sthosvd_csc",
    "tucker_rand_gaussian", "tucker_rand_colnorms", "tucker_rand_sample",
    "tucker_rand_gather", "tucker_rand_power", "tucker_rand_factor",
    "tucker_rand_ttm", "tucker_rand_status_string",
]

_DT = {torch.float64: TR_F64, torch.float32: TR_F32}


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype not in _DT:
        raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")
    return _DT[t.dtype]


def colmajor_empty(shape: Sequence[int], dtype=torch.float64, device="cuda") -> torch.Tensor:
    """Uninitialised tensor of ``shape`` with column-major strides."""
    shape = tuple(int(s) for s in shape)
    n = len(shape)
    return torch.empty(shape[::-1], dtype=dtype, device=device).permute(*range(n - 1, -1, -1))


def is_colmajor(t: torch.Tensor) -> bool:
    stride = 1
    for size, st in zip(t.shape, t.stride()):
        if size != 1 and st != stride:
            return False
        stride *= size
    return True


def to_device(a, dtype=None, device="cuda") -> torch.Tensor:
    """Copy a numpy array (any order) into a column-major device tensor."""
    src = torch.as_tensor(a)
    out = colmajor_empty(src.shape, dtype or src.dtype, device)
    out.copy_(src)
    return out


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream) -> c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _launch_stream(stream):
    """Context in which the step wrappers allocate: the launch stream, so that
    their fills precede the library's writes on it and a freed buffer is reused
    only after the work queued there."""
    return torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream())


def _i64arr(vals):
    arr = (c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def _flag_bits(flags) -> int:
    """tr_params.flags from an int or an iterable of names in _abi.FLAGS."""
    if isinstance(flags, int):
        return flags
    bits = 0
    for f in flags:
        bits |= _abi.FLAGS[f]
    return bits


def _params(dims, ranks, oversample, power, prob, samples, seed, precision, flags=0):
    N = len(dims)
    if len(ranks) != N:
        raise ValueError("ranks needs one entry per mode")
    p = _abi.TrParams()
    keep = [_i64arr(dims), _i64arr(ranks)]
    p.order = N
    p.dims = ctypes.cast(keep[0], ctypes.POINTER(c_int64))
    p.ranks = ctypes.cast(keep[1], ctypes.POINTER(c_int64))
    p.oversample = int(oversample)
    p.power = int(power)
    p.prob = PROB[prob] if isinstance(prob, str) else int(prob)
    if samples is not None:
        if len(samples) != N:
            raise ValueError("samples needs one entry per mode")
        keep.append(_i64arr(samples))
        p.samples = ctypes.cast(keep[2], ctypes.POINTER(c_int64))
    p.seed = int(seed) & ((1 << 64) - 1)
    p.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    p.flags = _flag_bits(flags)
    return p, keep


def tucker_rand_status_string(code: int) -> str:
    return _abi.status_string(code)


def tucker_rand_workspace_size(dims, ranks, oversample=10, power=1, prob="none",
                               samples=None, seed=0, dtype=torch.float32,
                               sthosvd=True, precision="native", flags=0) -> int:
    """Bytes of workspace tucker_rand_(s)thosvd needs (validates the arguments)."""
    p, _keep = _params(dims, ranks, oversample, power, prob, samples, seed, precision, flags)
    out = c_size_t(0)
    check("tucker_rand_workspace_size",
          lib().tucker_rand_workspace_size(byref(p), _DT[dtype], int(bool(sthosvd)), byref(out)))
    return out.value


class Timer:
    """Event-based kernel timer (tucker_rand_timer_*)."""

    def __init__(self, capacity=4096, classes=("colnorms", "ttm", "power", "factor",
                                               "sample", "gather", "gaussian")):
        mask = 0
        for c in classes:
            mask |= 1 << KC[c]
        h = c_void_p()
        check("tucker_rand_timer_create",
              lib().tucker_rand_timer_create(int(capacity), mask, byref(h)))
        self.handle = h

    def reset(self):
        check("tucker_rand_timer_reset", lib().tucker_rand_timer_reset(self.handle))

    def read(self, cls: str):
        """(total_ms, launches, mode0_ms, mode0_launches) for a kernel class."""
        t, n, t0, n0 = c_double(), c_int64(), c_double(), c_int64()
        check("tucker_rand_timer_read",
              lib().tucker_rand_timer_read(self.handle, KC[cls], byref(t), byref(n),
                                           byref(t0), byref(n0)))
        return t.value, n.value, t0.value, n0.value

    def close(self):
        if self.handle:
            lib().tucker_rand_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _decompose(fn_name, A, ranks, oversample, power, prob, samples, seed, precision,
               diag, timer, workspace, stream, out=None, flags=0):
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if not is_colmajor(A):
        raise ValueError("A must be column-major (use to_device / colmajor_empty)")
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    # every buffer is allocated and initialised on the launch stream, so the
    # fills are ordered before the library's writes and the caching allocator
    # reuses a freed buffer only after the work queued on that stream
    with torch.cuda.stream(st):
        return _decompose_on(fn_name, A, ranks, oversample, power, prob, samples, seed,
                             precision, diag, timer, workspace, st, out, flags)


def _decompose_on(fn_name, A, ranks, oversample, power, prob, samples, seed, precision,
                  diag, timer, workspace, stream, out, flags):
    dims = tuple(A.shape)
    N = len(dims)
    dt = _dtype_code(A)
    noalloc = fn_name == "tucker_rand_sthosvd_noalloc"
    sthosvd = fn_name != "tucker_rand_thosvd"
    p, keep = _params(dims, ranks, oversample, power, prob, samples, seed, precision, flags)
    need = c_size_t(0)
    check("tucker_rand_workspace_size",
          lib().tucker_rand_workspace_size(byref(p), dt, int(sthosvd), byref(need)))
    # (the allocation-free entry point rejects a workspace beyond its fixed
    # scratch itself, with TR_ENOMEM)
    if not noalloc and (workspace is None or workspace.numel() < need.value):
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=A.device)
    if out is None:
        Qs = [colmajor_empty((dims[n], ranks[n]), A.dtype, A.device) for n in range(N)]
        core = colmajor_empty(tuple(ranks), A.dtype, A.device)
    else:
        Qs, core = out
    qptrs = (c_void_p * N)(*[q.data_ptr() for q in Qs])
    info = {}
    dstruct = None
    if diag or timer is not None:
        dstruct = _abi.TrDiag()
        if diag:
            status = torch.zeros(1, dtype=torch.int32, device=A.device)
            info["status"] = status
            dstruct.status = status.data_ptr()
        if diag is True or diag == "norms":
            # ||A||^2, ||G||^2, RE of Eq. (8)
            info["norms"] = torch.zeros(3, dtype=torch.float64, device=A.device)
            dstruct.norms = info["norms"].data_ptr()
        if diag is True:
            # sketches and singular values for every mode
            s = [min(ranks[n] + oversample, dims[n]) for n in range(N)]
            cur = list(dims)
            I_n = []
            for n in range(N):
                I_n.append(cur[n])
                if sthosvd:
                    cur[n] = ranks[n]
            info["sketch"] = [torch.zeros((s[n], I_n[n]), dtype=torch.float64,
                                          device=A.device).t() for n in range(N)]
            info["sigma"] = [torch.zeros(s[n], dtype=torch.float64, device=A.device)
                             for n in range(N)]
            skp = (c_void_p * N)(*[t.data_ptr() for t in info["sketch"]])
            sgp = (c_void_p * N)(*[t.data_ptr() for t in info["sigma"]])
            keep += [skp, sgp]
            dstruct.sketch = ctypes.cast(skp, ctypes.POINTER(c_void_p))
            dstruct.sigma = ctypes.cast(sgp, ctypes.POINTER(c_void_p))
            if samples is not None and PROB.get(prob, prob) != 0:
                info["indices"] = [torch.full((int(samples[n]),), -1, dtype=torch.int64,
                                              device=A.device) for n in range(N)]
                info["scales"] = [torch.zeros(int(samples[n]), dtype=torch.float64,
                                              device=A.device) for n in range(N)]
                ip = (c_void_p * N)(*[t.data_ptr() for t in info["indices"]])
                sp = (c_void_p * N)(*[t.data_ptr() for t in info["scales"]])
                keep += [ip, sp]
                dstruct.indices = ctypes.cast(ip, ctypes.POINTER(c_void_p))
                dstruct.scales = ctypes.cast(sp, ctypes.POINTER(c_void_p))
        if timer is not None:
            dstruct.timer = timer.handle
    fn = getattr(lib(), fn_name)
    dptr = byref(dstruct) if dstruct is not None else None
    if noalloc:
        rc = fn(byref(p), dt, c_void_p(A.data_ptr()), qptrs, c_void_p(core.data_ptr()), dptr,
                _stream(stream))
    else:
        rc = fn(byref(p), dt, c_void_p(A.data_ptr()), qptrs, c_void_p(core.data_ptr()),
                c_void_p(workspace.data_ptr()), c_size_t(workspace.numel()), dptr,
                _stream(stream))
    check(fn_name, rc)
    return Qs, core, info


def tucker_rand_thosvd(A: torch.Tensor, ranks, oversample=10, power=1, prob="none",
                       samples=None, seed=0, precision="native", diag=False, timer=None,
                       workspace=None, stream=None, out=None, flags=0):
    """Randomized T-HOSVD (Alg. 1 / Alg. 4).  Returns (Q list, core, diag dict)."""
    return _decompose("tucker_rand_thosvd", A, ranks, oversample, power, prob, samples,
                      seed, precision, diag, timer, workspace, stream, out, flags)


def tucker_rand_sthosvd(A: torch.Tensor, ranks, oversample=10, power=1, prob="none",
                        samples=None, seed=0, precision="native", diag=False, timer=None,
                        workspace=None, stream=None, out=None, flags=0):
    """Randomized ST-HOSVD (Alg. 2 / Alg. 5).  Returns (Q list, core, diag dict)."""
    return _decompose("tucker_rand_sthosvd", A, ranks, oversample, power, prob, samples,
                      seed, precision, diag, timer, workspace, stream, out, flags)


def tucker_rand_sthosvd_noalloc(A: torch.Tensor, ranks, oversample=10, power=1, prob="none",
                                samples=None, seed=0, precision="native", diag=False,
                                timer=None, stream=None, out=None, flags=0):
    """Randomized ST-HOSVD whose library call allocates nothing: the workspace is
    the library's fixed device scratch (at most ``_abi.NOALLOC_SCRATCH_BYTES``).
    Calls that overlap in time on one GPU race.  Pass ``out=(Qs, core)`` (and no
    ``diag``) for a call with no allocation on the Python side either."""
    return _decompose("tucker_rand_sthosvd_noalloc", A, ranks, oversample, power, prob,
                      samples, seed, precision, diag, timer, None, stream, out, flags)


def tucker_rand_sthosvd_csc(colptr: torch.Tensor, rowidx: torch.Tensor, vals: torch.Tensor,
                            dims, ranks, oversample=10, power=1, prob="nearly_optimal",
                            samples=None, seed=0, diag=False, workspace=None, stream=None,
                            out=None):
    """Randomized ST-HOSVD with sampled products (Alg. 5) of a sparse tensor of
    shape ``dims`` given as the compressed sparse columns of its mode-1
    unfolding: ``colptr`` int64 [J_1 + 1], ``rowidx`` int32 [nnz] (rows
    increasing within a column), ``vals`` [nnz] float32 or float64, all on
    the device.  Returns (Q list, core, diag dict) as tucker_rand_sthosvd."""
    for t, dt in ((colptr, torch.int64), (rowidx, torch.int32)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("colptr must be contiguous device int64, rowidx device int32")
    if not vals.is_cuda or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous device tensor")
    dims = tuple(int(d) for d in dims)
    N = len(dims)
    if colptr.numel() != math.prod(dims[1:]) + 1 or rowidx.numel() != vals.numel():
        raise ValueError("colptr needs J_1 + 1 entries and rowidx one per value")
    dt = _dtype_code(vals)
    st = stream if stream is not None else torch.cuda.current_stream(vals.device)
    p, keep = _params(dims, ranks, oversample, power, prob, samples, seed, "native")
    need = c_size_t(0)
    check("tucker_rand_workspace_size",
          lib().tucker_rand_workspace_size(byref(p), dt, 1, byref(need)))
    with torch.cuda.stream(st):
        if workspace is None:
            workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=vals.device)
        if out is None:
            Qs = [colmajor_empty((dims[n], ranks[n]), vals.dtype, vals.device) for n in range(N)]
            core = colmajor_empty(tuple(ranks), vals.dtype, vals.device)
        else:
            Qs, core = out
        info, dstruct = {}, None
        if diag:
            dstruct = _abi.TrDiag()
            info["status"] = torch.zeros(1, dtype=torch.int32, device=vals.device)
            dstruct.status = info["status"].data_ptr()
            info["norms"] = torch.zeros(3, dtype=torch.float64, device=vals.device)
            dstruct.norms = info["norms"].data_ptr()
    qptrs = (c_void_p * N)(*[q.data_ptr() for q in Qs])
    rc = lib().tucker_rand_sthosvd_csc(byref(p), dt, vals.numel(), c_void_p(colptr.data_ptr()),
                                       c_void_p(rowidx.data_ptr()), c_void_p(vals.data_ptr()),
                                       qptrs, c_void_p(core.data_ptr()),
                                       c_void_p(workspace.data_ptr()), c_size_t(workspace.numel()),
                                       byref(dstruct) if dstruct is not None else None,
                                       _stream(st))
    check("tucker_rand_sthosvd_csc", rc)
    del keep
    return Qs, core, info


class BatchRequest:
    """One request of tucker_rand_sthosvd_batch: a column-major device tensor
    and its parameters (sampled products, Alg. 5)."""

    def __init__(self, A, ranks, samples, oversample=10, power=1, prob="nearly_optimal",
                 seed=0):
        self.A, self.ranks, self.samples = A, tuple(ranks), tuple(samples)
        self.oversample, self.power, self.prob, self.seed = oversample, power, prob, seed

    def params(self, dims=None):
        return _params(tuple(dims if dims is not None else self.A.shape), self.ranks,
                       self.oversample, self.power, self.prob, self.samples, self.seed,
                       "native")


def _batch_params(reqs, dims=None):
    ps, keep = [], []
    for i, r in enumerate(reqs):
        p, k = r.params(None if dims is None else dims[i])
        ps.append(p)
        keep.append(k)
    arr = (ctypes.POINTER(_abi.TrParams) * len(ps))(*[ctypes.pointer(p) for p in ps])
    return arr, (ps, keep)


def tucker_rand_batch_workspace_size(reqs, dtype=torch.float32, dims=None) -> int:
    """Bytes of workspace tucker_rand_sthosvd_batch needs for these requests
    (``dims``: their shapes, when the tensors are not given yet)."""
    arr, _keep = _batch_params(reqs, dims)
    out = c_size_t(0)
    check("tucker_rand_batch_workspace_size",
          lib().tucker_rand_batch_workspace_size(len(reqs), arr, _DT[dtype], byref(out)))
    return out.value


def tucker_rand_sthosvd_batch(reqs, workspace=None, stream=None, status=True, out=None):
    """Randomized ST-HOSVD with sampled products (Alg. 5) for a batch of
    requests of one order and dtype, every stage one grouped launch.  Returns
    (list of Q lists, list of cores, status tensor [nreq] or None).  The
    descriptor copy synchronises the host with the stream's earlier work."""
    if not reqs:
        raise ValueError("empty batch")
    A0 = reqs[0].A
    dt = _dtype_code(A0)
    for r in reqs:
        if not r.A.is_cuda or not is_colmajor(r.A):
            raise ValueError("every A must be a column-major device tensor")
        if r.A.dtype != A0.dtype or r.A.dim() != A0.dim():
            raise ValueError("every request needs the same dtype and order")
    st = stream if stream is not None else torch.cuda.current_stream(A0.device)
    arr, keep = _batch_params(reqs)
    need = c_size_t(0)
    check("tucker_rand_batch_workspace_size",
          lib().tucker_rand_batch_workspace_size(len(reqs), arr, dt, byref(need)))
    with torch.cuda.stream(st):
        # (a workspace the caller passes is used as it is: the library rejects
        # one that is too small)
        if workspace is None:
            workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=A0.device)
        if out is None:
            Qs = [[colmajor_empty((r.A.shape[n], r.ranks[n]), r.A.dtype, r.A.device)
                   for n in range(r.A.dim())] for r in reqs]
            cores = [colmajor_empty(r.ranks, r.A.dtype, r.A.device) for r in reqs]
        else:
            Qs, cores = out
        stat = torch.zeros(len(reqs), dtype=torch.int32, device=A0.device) if status else None
    nreq, N = len(reqs), A0.dim()
    qrows = [(c_void_p * N)(*[q.data_ptr() for q in Qs[i]]) for i in range(nreq)]
    qtab = (ctypes.POINTER(c_void_p) * nreq)(
        *[ctypes.cast(q, ctypes.POINTER(c_void_p)) for q in qrows])
    atab = (c_void_p * nreq)(*[r.A.data_ptr() for r in reqs])
    ctab = (c_void_p * nreq)(*[c.data_ptr() for c in cores])
    check("tucker_rand_sthosvd_batch",
          lib().tucker_rand_sthosvd_batch(nreq, arr, dt, atab, qtab, ctab,
                                          c_void_p(workspace.data_ptr()),
                                          c_size_t(workspace.numel()), _ptr(stat),
                                          _stream(st)))
    del keep
    return Qs, cores, stat


def tucker_rand_adaptive(A: torch.Tensor, tol: float, max_ranks, oversample=10, power=1,
                         prob="none", samples=None, seed=0, sthosvd=True, relative=True,
                         precision="native", flags=0, diag=False, stream=None):
    """Fixed-precision Problem 2: ranks mu_n <= max_ranks[n] and factors with
    ||A - A^||_F <= tol (times ||A||_F when ``relative``), by the rule of
    tucker_rand_adaptive in include/tucker_rand.h.  Returns
    (Q list (I_n x mu_n views), core (mu view), ranks, bound, diag dict);
    ``bound`` is the certified bound on ||A - A^||_F.  Synchronises the stream."""
    if not A.is_cuda or not is_colmajor(A):
        raise ValueError("A must be a column-major device tensor")
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    with torch.cuda.stream(st):
        dims = tuple(A.shape)
        N = len(dims)
        dt = _dtype_code(A)
        bits = _flag_bits(flags) | _abi.FLAGS["related_form"]
        p, keep = _params(dims, max_ranks, oversample, power, prob, samples, seed, precision,
                          bits)
        need = c_size_t(0)
        check("tucker_rand_workspace_size",
              lib().tucker_rand_workspace_size(byref(p), dt, int(bool(sthosvd)), byref(need)))
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=A.device)
        Qb = [colmajor_empty((dims[n], max_ranks[n]), A.dtype, A.device) for n in range(N)]
        cb = torch.empty(int(math.prod(max_ranks)), dtype=A.dtype, device=A.device)
        qptrs = (c_void_p * N)(*[q.data_ptr() for q in Qb])
        info, dptr = {}, None
        if diag:
            d = _abi.TrDiag()
            info["status"] = torch.zeros(1, dtype=torch.int32, device=A.device)
            info["norms"] = torch.zeros(3, dtype=torch.float64, device=A.device)
            d.status = info["status"].data_ptr()
            d.norms = info["norms"].data_ptr()
            dptr = byref(d)
        ranks = (c_int64 * N)()
        bound = c_double(0.0)
        check("tucker_rand_adaptive",
              lib().tucker_rand_adaptive(byref(p), dt, int(bool(sthosvd)), float(tol),
                                         int(bool(relative)), c_void_p(A.data_ptr()), qptrs,
                                         c_void_p(cb.data_ptr()), c_void_p(ws.data_ptr()),
                                         c_size_t(ws.numel()), ranks, byref(bound), dptr,
                                         _stream(st)))
        mus = [int(r) for r in ranks]
        Qs = [Qb[n][:, :mus[n]] for n in range(N)]
        strides, acc = [], 1
        for m in mus:
            strides.append(acc)
            acc *= m
        core = cb.as_strided(tuple(mus), tuple(strides))
        return Qs, core, mus, bound.value, info


def _view3(X: torch.Tensor, L, I, R):
    if not X.is_cuda or not X.is_contiguous() and not is_colmajor(X):
        raise ValueError("X must be a dense device tensor")
    if X.numel() != L * I * R:
        raise ValueError("L*I*R does not match the tensor size")


def tucker_rand_gaussian(I: int, s: int, mode: int, seed: int, device="cuda", stream=None):
    """G_n (I x s, float64, column-major) from the library's Philox stream."""
    with _launch_stream(stream):
        G = colmajor_empty((I, s), torch.float64, device)
        check("tucker_rand_gaussian",
              lib().tucker_rand_gaussian(I, s, mode, int(seed) & ((1 << 64) - 1),
                                         c_void_p(G.data_ptr()), _stream(stream)))
        return G


def tucker_rand_colnorms(X: torch.Tensor, L: int, I: int, R: int, stream=None):
    """(norms float64 [L*R], max bit pattern as int64 tensor [1])."""
    with _launch_stream(stream):
        _view3(X, L, I, R)
        norms = torch.empty(L * R, dtype=torch.float64, device=X.device)
        mb = torch.zeros(1, dtype=torch.int64, device=X.device)
        check("tucker_rand_colnorms",
              lib().tucker_rand_colnorms(_dtype_code(X), c_void_p(X.data_ptr()), L, I, R,
                                         c_void_p(norms.data_ptr()), c_void_p(mb.data_ptr()),
                                         _stream(stream)))
        return norms, mb


def tucker_rand_sample(norms: Optional[torch.Tensor], J: int, T: int, prob: str, seed: int,
                       mode: int, device="cuda", stream=None):
    """(idx int64 [T], scale float64 [T], status int32 [1])."""
    with _launch_stream(stream):
        ws = torch.empty(max(1, lib().tucker_rand_sample_workspace_size(J)), dtype=torch.uint8,
                         device=device)
        idx = torch.empty(T, dtype=torch.int64, device=device)
        scale = torch.empty(T, dtype=torch.float64, device=device)
        status = torch.zeros(1, dtype=torch.int32, device=device)
        check("tucker_rand_sample",
              lib().tucker_rand_sample(_ptr(norms), J, T, PROB[prob], int(seed) & ((1 << 64) - 1),
                                       mode, c_void_p(idx.data_ptr()), c_void_p(scale.data_ptr()),
                                       c_void_p(ws.data_ptr()), c_size_t(ws.numel()),
                                       c_void_p(status.data_ptr()), _stream(stream)))
        return idx, scale, status


def tucker_rand_gather(X: torch.Tensor, L: int, I: int, R: int, idx: torch.Tensor,
                       stream=None):
    """C' = A_(n)(:, idx) without rescale, I x T column-major (X's dtype)."""
    with _launch_stream(stream):
        _view3(X, L, I, R)
        T = idx.numel()
        Cp = colmajor_empty((I, T), X.dtype, X.device)
        check("tucker_rand_gather",
              lib().tucker_rand_gather(_dtype_code(X), c_void_p(X.data_ptr()), L, I, R,
                                       c_void_p(idx.data_ptr()), T, c_void_p(Cp.data_ptr()),
                                       _stream(stream)))
        return Cp


def tucker_rand_power(X: torch.Tensor, L: int, I: int, R: int, G: torch.Tensor, q: int,
                      colweight: Optional[torch.Tensor] = None, stream=None):
    """C = (M D M^T)^q G for the mode-n unfolding M of the L x I x R view of X."""
    with _launch_stream(stream):
        _view3(X, L, I, R)
        if not is_colmajor(G) or G.dtype != torch.float64:
            raise ValueError("G must be column-major float64")
        s = G.shape[1]
        C = colmajor_empty((I, s), torch.float64, X.device)
        wsn = lib().tucker_rand_power_workspace_size(_dtype_code(X), L, I, R, s)
        ws = torch.empty(max(1, wsn), dtype=torch.uint8, device=X.device)
        check("tucker_rand_power",
              lib().tucker_rand_power(_dtype_code(X), c_void_p(X.data_ptr()), L, I, R,
                                      _ptr(colweight), q, c_void_p(G.data_ptr()), s,
                                      c_void_p(C.data_ptr()), c_void_p(ws.data_ptr()),
                                      c_size_t(ws.numel()), _stream(stream)))
        return C


def tucker_rand_factor(C: torch.Tensor, mu: int, stream=None):
    """(Q I x mu float64 column-major, sigma [s]) from a sketch C (I x s float64)."""
    with _launch_stream(stream):
        if not is_colmajor(C) or C.dtype != torch.float64:
            raise ValueError("C must be column-major float64")
        I, s = C.shape
        Q = colmajor_empty((I, mu), torch.float64, C.device)
        sig = torch.empty(s, dtype=torch.float64, device=C.device)
        wsn = lib().tucker_rand_factor_workspace_size(I, s, mu)
        ws = torch.empty(max(1, wsn), dtype=torch.uint8, device=C.device)
        check("tucker_rand_factor",
              lib().tucker_rand_factor(c_void_p(C.data_ptr()), I, s, mu, c_void_p(Q.data_ptr()),
                                       c_void_p(sig.data_ptr()), c_void_p(ws.data_ptr()),
                                       c_size_t(ws.numel()), _stream(stream)))
        return Q, sig


def tucker_rand_ttm(X: torch.Tensor, L: int, I: int, R: int, Q: torch.Tensor,
                    out_dtype=torch.float64, stream=None):
    """Y = X x_n Q^T as a flat column-major L x mu x R buffer (out_dtype)."""
    with _launch_stream(stream):
        _view3(X, L, I, R)
        if not is_colmajor(Q) or Q.dtype != torch.float64:
            raise ValueError("Q must be column-major float64")
        mu = Q.shape[1]
        wsn = lib().tucker_rand_ttm_workspace_size(L, I, R, mu)
        ws = torch.empty(max(1, wsn), dtype=torch.uint8, device=X.device)
        Y = torch.empty(L * mu * R, dtype=out_dtype, device=X.device)
        check("tucker_rand_ttm",
              lib().tucker_rand_ttm(_dtype_code(X), c_void_p(X.data_ptr()), L, I, R,
                                    c_void_p(Q.data_ptr()), mu, _DT[out_dtype],
                                    c_void_p(Y.data_ptr()), c_void_p(ws.data_ptr()),
                                    c_size_t(ws.numel()), _stream(stream)))
        return Y

