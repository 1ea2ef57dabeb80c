"""Continuous-batching server for randomized ST-HOSVD requests (Alg. 5).

Requests (a tensor plus its multilinear rank, sample counts and seed) arrive
over time.  The server admits an arrived request as soon as a slot is free and
its HBM footprint -- workspace, factors and core, plus the device copy of the
tensor when it arrives in host memory -- fits the budget beside the requests
already running; nothing waits for a batch to fill.  Each slot owns a HIP
stream, so admitted requests run concurrently and one request's latency-bound
steps (sampler, small factorizations) overlap another's HBM sweeps.  Requests
are taken in arrival order; one that does not fit yet does not block the next
few that do (bounded look-ahead).  Every request runs the same library call
as a lone request with the same arguments, and the kernels are deterministic
(fixed reduction orders, no floating-point atomics), so each result is
bitwise the same alone and in the mix.

Latency is device completion time minus arrival time on one timeline: the
host clock at a synchronized reference event, plus the device time from that
event to the request's completion event.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

GIB = 1 << 30


@dataclasses.dataclass
class Request:
    rid: int
    X: object                         # column-major torch tensor, on the device or pinned host
    ranks: tuple
    samples: Optional[tuple] = None
    oversample: int = 10
    power: int = 1
    prob: str = "nearly_optimal"
    seed: int = 0
    arrival: float = 0.0              # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    completed: float = float("nan")
    footprint: int = 0
    slot: int = -1
    status: int = 0
    factors: object = None            # list of device tensors
    core: object = None               # device tensor

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def percentile(xs: Sequence[float], p: float) -> float:
    """Nearest-rank percentile."""
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(np.ceil(p / 100.0 * len(xs))) - 1))
    return xs[k]


def pinned_colmajor(A) -> "torch.Tensor":
    """Copy of the array A in page-locked host memory, column-major, float32."""
    import torch
    shape = tuple(A.shape)
    n = int(np.prod(shape))
    buf = torch.empty(n, dtype=torch.float32, pin_memory=True)
    buf.numpy()[:] = np.ravel(np.asarray(A, dtype=np.float32), order="F")
    strides, st = [], 1
    for d in shape:
        strides.append(st)
        st *= d
    return buf.as_strided(shape, tuple(strides))


class GpuBackend:
    """Runs each request through tucker_rand_sthosvd on its slot's stream."""

    def __init__(self, slots: int):
        import torch
        from . import colmajor_empty, tucker_rand_sthosvd, tucker_rand_workspace_size
        self.torch = torch
        self._colmajor_empty = colmajor_empty
        self._sthosvd = tucker_rand_sthosvd
        self._ws_size = tucker_rand_workspace_size
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def footprint(self, req: Request) -> int:
        """Device bytes the request holds while it runs."""
        X = req.X
        esz = X.element_size()
        ws = self._ws_size(tuple(X.shape), req.ranks, req.oversample, req.power, req.prob,
                           req.samples, req.seed, X.dtype, sthosvd=True)
        out = sum(X.shape[n] * req.ranks[n] for n in range(X.dim())) + int(np.prod(req.ranks))
        staged = 0 if X.is_cuda else X.numel() * esz
        return int(staged + ws + out * esz + 4)

    def launch(self, req: Request, slot: int):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            X = req.X
            if not X.is_cuda:
                host = X
                X = self._colmajor_empty(tuple(host.shape), host.dtype)
                X.copy_(host, non_blocking=True)
            Qs, core, info = self._sthosvd(X, req.ranks, req.oversample, req.power, req.prob,
                                           req.samples, req.seed, diag="status", stream=st)
            done = torch.cuda.Event(enable_timing=True)
            done.record(st)
        # X, the workspace and the outputs were allocated on `st`, so the
        # caching allocator reuses their blocks only for later work on `st`.
        return {"X": X, "Qs": Qs, "core": core, "status": info["status"], "done": done}

    def poll(self, h) -> bool:
        return h["done"].query()

    def reference(self):
        torch = self.torch
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        torch.cuda.synchronize()
        return ref, time.perf_counter()

    def completion_time(self, h, ref) -> float:
        """Host-clock time at which the request's last kernel finished."""
        return ref[1] + ref[0].elapsed_time(h["done"]) * 1e-3

    def finish(self, h, res: Result):
        res.status = int(h["status"].item())
        res.factors = h["Qs"]
        res.core = h["core"]


class Server:
    """Admission by free slot and HBM footprint, in arrival order."""

    def __init__(self, backend, slots: int = 8, hbm_budget: int = 16 * GIB,
                 lookahead: int = 8):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.backend = backend
        self.slots = slots
        self.budget = int(hbm_budget)
        self.lookahead = max(1, int(lookahead))

    def run(self, requests: List[Request], clock: Optional[Callable[[], float]] = None,
            idle: Optional[Callable[[], None]] = None) -> List[Result]:
        """Serve the requests (arrival times in seconds after the start).

        Returns one Result per request, in rid order.  A request whose
        footprint exceeds the whole budget is rejected up front (ValueError).
        """
        be = self.backend
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        fps = {r.rid: be.footprint(r) for r in reqs}
        for r in reqs:
            if fps[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {fps[r.rid]} B of HBM, "
                                 f"more than the budget of {self.budget} B")
        ref = be.reference()
        t0 = ref[1]
        if clock is None:
            def clock():
                return time.perf_counter() - t0
        pending = list(reqs)
        active = {}                   # slot -> (request, handle, Result)
        used = 0
        self.peak_used = 0
        results = {}
        while pending or active:
            # completions
            for slot in list(active):
                r, h, res = active[slot]
                if be.poll(h):
                    res.completed = be.completion_time(h, ref) - t0
                    be.finish(h, res)
                    results[r.rid] = res
                    used -= res.footprint
                    del active[slot]
            # admissions: arrived requests in arrival order, bounded look-ahead
            now = clock()
            free = [s for s in range(self.slots) if s not in active]
            i = 0
            while free and i < min(len(pending), self.lookahead):
                r = pending[i]
                if r.arrival > now:
                    break
                if used + fps[r.rid] <= self.budget:
                    slot = free.pop(0)
                    res = Result(r.rid, r.arrival, now, footprint=fps[r.rid], slot=slot)
                    active[slot] = (r, be.launch(r, slot), res)
                    used += fps[r.rid]
                    self.peak_used = max(self.peak_used, used)
                    pending.pop(i)
                else:
                    i += 1
            if idle is not None:
                idle()
            elif not active and pending and pending[0].arrival > clock():
                time.sleep(min(1e-3, max(0.0, pending[0].arrival - clock())))
        return [results[r.rid] for r in sorted(reqs, key=lambda r: r.rid)]


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds) of n requests of a Poisson stream of `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def summarize(results: List[Result]) -> dict:
    lat = [r.latency for r in results]
    span = max(r.completed for r in results) - min(r.arrival for r in results)
    return {"requests": len(results),
            "p50_ms": round(1e3 * percentile(lat, 50), 4),
            "p99_ms": round(1e3 * percentile(lat, 99), 4),
            "mean_ms": round(1e3 * float(np.mean(lat)), 4),
            "throughput_rps": round(len(results) / span, 2) if span > 0 else None}
