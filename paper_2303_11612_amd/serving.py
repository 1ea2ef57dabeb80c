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


class GroupedBackend:
    """Runs a group of admitted requests through one tucker_rand_sthosvd_batch
    call on the slot's stream: every stage of every mode is one launch for the
    whole group.  A request's result is bitwise the same in any group (and
    differs from GpuBackend's only by float64 rounding: the grouped kernels
    sum in other orders)."""

    grouped = True

    def __init__(self, slots: int, max_group: int = 64):
        import torch
        from . import (BatchRequest, colmajor_empty, tucker_rand_batch_workspace_size,
                       tucker_rand_sthosvd_batch)
        self.torch = torch
        self.max_group = max(1, int(max_group))
        self._colmajor_empty = colmajor_empty
        self._breq = BatchRequest
        self._ws_size = tucker_rand_batch_workspace_size
        self._batch = tucker_rand_sthosvd_batch
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def _request(self, req: Request, X):
        return self._breq(X, req.ranks, req.samples, req.oversample, req.power, req.prob,
                          req.seed)

    def compatible(self, a: Request, b: Request) -> bool:
        """Requests that can share a group: the same order and dtype."""
        return a.X.dim() == b.X.dim() and a.X.dtype == b.X.dtype

    def footprint(self, req: Request) -> int:
        """Device bytes the request holds while its group runs (its workspace
        alone bounds its share of a group's: the per-request regions are the
        same and the descriptor area grows linearly)."""
        X = req.X
        esz = X.element_size()
        ws = self._ws_size([self._request(req, None)], X.dtype, dims=[tuple(X.shape)])
        out = sum(X.shape[n] * req.ranks[n] for n in range(X.dim())) + int(np.prod(req.ranks))
        staged = 0 if X.is_cuda else X.numel() * esz
        return int(staged + ws + out * esz + 4)

    def launch_group(self, reqs: List[Request], slot: int):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            Xs = []
            for req in reqs:
                X = req.X
                if not X.is_cuda:
                    host = X
                    X = self._colmajor_empty(tuple(host.shape), host.dtype)
                    X.copy_(host, non_blocking=True)
                Xs.append(X)
            Qs, cores, stat = self._batch([self._request(r, X) for r, X in zip(reqs, Xs)],
                                          stream=st)
            done = torch.cuda.Event(enable_timing=True)
            done.record(st)
        return {"X": Xs, "Qs": Qs, "cores": cores, "status": stat, "done": done}

    def poll(self, h) -> bool:
        return h["done"].query()

    reference = GpuBackend.reference
    completion_time = GpuBackend.completion_time

    def finish_group(self, h, results: List[Result]):
        stat = h["status"].cpu().tolist()
        for i, res in enumerate(results):
            res.status = int(stat[i])
            res.factors = h["Qs"][i]
            res.core = h["cores"][i]


class Server:
    """Admission by free slot and HBM footprint, in arrival order.

    With a grouped backend (``backend.grouped``) a free slot takes every
    arrived request that fits -- up to ``backend.max_group``, compatible with
    the first -- as one group; otherwise one request per slot."""

    def __init__(self, backend, slots: int = 8, hbm_budget: int = 16 * GIB,
                 lookahead: int = 8):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.backend = backend
        self.slots = slots
        self.budget = int(hbm_budget)
        self.lookahead = max(1, int(lookahead))
        self.group_sizes = []

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
        grouped = getattr(be, "grouped", False)
        gmax = be.max_group if grouped else 1
        pending = list(reqs)
        active = {}                   # slot -> (handle, [Result])
        used = 0
        self.peak_used = 0
        self.group_sizes = []
        results = {}
        while pending or active:
            # completions
            for slot in list(active):
                h, group = active[slot]
                if be.poll(h):
                    t_done = be.completion_time(h, ref) - t0
                    if grouped:
                        be.finish_group(h, group)
                    else:
                        be.finish(h, group[0])
                    for res in group:
                        res.completed = t_done
                        results[res.rid] = res
                        used -= res.footprint
                    del active[slot]
            # admissions: arrived requests in arrival order, bounded look-ahead
            # (per group member)
            now = clock()
            free = [s for s in range(self.slots) if s not in active]
            while free and pending and pending[0].arrival <= now:
                take, i = [], 0
                budget_left = self.budget - used
                while len(take) < gmax and i < len(pending) and \
                        i < len(take) + self.lookahead:
                    r = pending[i]
                    if r.arrival > now:
                        break
                    if fps[r.rid] <= budget_left and \
                            (not take or be.compatible(pending[take[0]], r)):
                        take.append(i)
                        budget_left -= fps[r.rid]
                    i += 1
                if not take:
                    break
                slot = free.pop(0)
                group_reqs = [pending[i] for i in take]
                for i in reversed(take):
                    pending.pop(i)
                group = [Result(r.rid, r.arrival, now, footprint=fps[r.rid], slot=slot)
                         for r in group_reqs]
                h = be.launch_group(group_reqs, slot) if grouped else be.launch(group_reqs[0],
                                                                                slot)
                active[slot] = (h, group)
                used += sum(res.footprint for res in group)
                self.peak_used = max(self.peak_used, used)
                self.group_sizes.append(len(group))
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
