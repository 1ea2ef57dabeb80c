"""Continuous batching on the GPU: every result is bitwise the same alone and
in the mix, and matches the FP64 oracle (float32 bar 1e-4).  The grouped
server (GroupedBackend: admitted requests run as one tucker_rand_sthosvd_batch
call) gives each request bitwise the result of that request alone in a batch,
whatever the grouping.

Requests are the serving stream's (modes 32..384, ranks 4..24, T_n = 4 mu_n,
nearly-optimal sampling, q = 1, K = 10).  "Alone" runs each request by itself
on one slot; "mix" runs all of them over four streams at once, and a third
run adds an HBM budget that admits only some at a time, so admission, stream
assignment and overlap all differ from the lone runs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2303_11612_amd as tr
from paper_2303_11612_amd.serving import (GpuBackend, GroupedBackend, Request, Server,
                                          pinned_colmajor)

pytestmark = pytest.mark.gpu

NREQ = 10


@pytest.fixture(scope="module")
def stream_requests():
    out = []
    for rid in range(NREQ):
        A, ranks, samples = synth.serving_request(rid)
        out.append((A, ranks, samples))
    return out


def _requests(stream_requests, source, arrivals=None):
    reqs = []
    for rid, (A, ranks, samples) in enumerate(stream_requests):
        X = tr.to_device(A) if source == "device" else pinned_colmajor(A)
        reqs.append(Request(rid, X, ranks, samples, seed=rid,
                            arrival=0.0 if arrivals is None else float(arrivals[rid])))
    return reqs


def _np(t):
    return t.detach().cpu().numpy()


def _outputs(results):
    torch.cuda.synchronize()
    return [([_np(Q) for Q in r.factors], _np(r.core)) for r in results]


@pytest.fixture(scope="module")
def alone(stream_requests):
    outs = []
    for req in _requests(stream_requests, "device"):
        res = Server(GpuBackend(1), slots=1).run([req])
        assert res[0].status == 0
        outs += _outputs(res)
    return outs


def _same(a, b):
    for (Qa, ca), (Qb, cb) in zip(a, b):
        for x, y in zip(Qa, Qb):
            assert np.array_equal(x, y)
        assert np.array_equal(ca, cb)


@pytest.mark.parametrize("source", ["device", "host"])
def test_mix_equals_alone(stream_requests, alone, source):
    res = Server(GpuBackend(4), slots=4).run(_requests(stream_requests, source))
    assert all(r.status == 0 for r in res)
    assert len({r.slot for r in res}) > 1
    _same(_outputs(res), alone)


def test_budget_bound_mix_equals_alone(stream_requests, alone):
    reqs = _requests(stream_requests, "host", arrivals=np.arange(NREQ) * 2e-4)
    be = GpuBackend(4)
    fps = [be.footprint(r) for r in reqs]
    budget = int(1.2 * max(fps))          # forces admission to wait for HBM
    srv = Server(be, slots=4, hbm_budget=budget)
    res = srv.run(reqs)
    assert srv.peak_used <= budget
    assert all(r.status == 0 for r in res)
    assert all(r.admitted >= r.arrival and r.completed > r.admitted for r in res)
    _same(_outputs(res), alone)


def test_mix_matches_oracle(stream_requests, alone):
    for rid in range(3):
        A, ranks, samples = stream_requests[rid]
        Qo, co, infos = oracle.rand_sthosvd(A.astype(np.float64), ranks, 10, 1,
                                            "nearly_optimal", samples, rid)
        Qg, cg = alone[rid]
        for n in range(3):
            sig = infos[n]["sigma"]
            gaps = [(sig[c] - sig[c + 1]) / sig[0] for c in range(ranks[n])
                    if c + 1 < len(sig)]
            if min(gaps, default=1.0) < 1e-6:
                Pg, Po = Qg[n] @ Qg[n].T, Qo[n] @ Qo[n].T
                assert np.linalg.norm(Pg - Po, 2) <= 1e-4, (rid, n)
            else:
                err = np.linalg.norm(Qg[n] - Qo[n]) / np.linalg.norm(Qo[n])
                assert err <= 1e-4, (rid, n, err)
        A64 = A.astype(np.float64)
        re_o = oracle.relative_error(A64, co, Qo)
        re_g = oracle.relative_error(A64, cg.astype(np.float64), [Q.astype(np.float64) for Q in Qg])
        assert abs(re_g - re_o) <= 1e-4 * max(re_o, 1e-3), (rid, re_g, re_o)


@pytest.fixture(scope="module")
def alone_grouped(stream_requests):
    outs = []
    for req in _requests(stream_requests, "device"):
        res = Server(GroupedBackend(1, 1), slots=1).run([req])
        assert res[0].status == 0
        outs += _outputs(res)
    return outs


@pytest.mark.parametrize("source", ["device", "host"])
def test_grouped_mix_equals_alone(stream_requests, alone_grouped, source):
    srv = Server(GroupedBackend(2, 4), slots=2)
    res = srv.run(_requests(stream_requests, source))
    assert all(r.status == 0 for r in res)
    assert max(srv.group_sizes) > 1 and sum(srv.group_sizes) == NREQ
    _same(_outputs(res), alone_grouped)


def test_grouped_budget_and_arrivals(stream_requests, alone_grouped):
    reqs = _requests(stream_requests, "host", arrivals=np.arange(NREQ) * 2e-4)
    be = GroupedBackend(3, 3)
    budget = int(2.5 * max(be.footprint(r) for r in reqs))
    srv = Server(be, slots=3, hbm_budget=budget)
    res = srv.run(reqs)
    assert srv.peak_used <= budget
    assert all(r.status == 0 and r.admitted >= r.arrival and r.completed > r.admitted
               for r in res)
    _same(_outputs(res), alone_grouped)


def test_grouped_close_to_per_request_driver(alone, alone_grouped, stream_requests):
    """The grouped kernels sum in other orders than tucker_rand_sthosvd: the
    two results agree to float32 output rounding (both are within the float32
    bar of the oracle)."""
    for (Qa, ca), (Qb, cb) in zip(alone, alone_grouped):
        for x, y in zip(Qa, Qb):
            x64, y64 = x.astype(np.float64), y.astype(np.float64)
            d = max(np.linalg.norm(x64 - y64 @ (y64.T @ x64), 2),
                    np.linalg.norm(y64 - x64 @ (x64.T @ y64), 2))
            assert d <= 1e-4
