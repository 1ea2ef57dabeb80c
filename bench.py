#!/usr/bin/env python3
"""Benchmark of the randomized Tucker hot path on one MI355X.

Workload (one step = one whole decomposition, inputs resident in HBM):
randomized ST-HOSVD with column-sampled approximate products (Alg. 5) of a
400 x 400 x 400 float32 tensor (superdiagonal core with singular values 0.5^k,
k < 10, orthonormal Gaussian factors, 1e-4 relative Gaussian noise), ranks
(10, 10, 10), oversampling K = 10, q = 1, T_n = 4000 columns per mode drawn
with nearly-optimal probabilities p_j ~ ||A_(n)(:, j)||^2.

Prints one JSON line.  ``value`` is decompositions per second over K steps
with nothing recorded between them; a second pass of K steps gives the
per-step latency (event pair per step) and a third the per-kernel durations
(HIP events on the launch stream around every kernel class).  ``roofline``
is the dominant kernel class by device time per step (its algorithmic bytes
or flops per launch over its average launch time); ``sweep_roofline`` the
longer of the two mode-1 sweeps over the whole tensor (column norms, shrink).
RE comes from the library's float64 norms (Eq. (8)) and is cross-checked by
an explicit float64 reconstruction.  The CPU baseline is the FP64 oracle on
the same input and seed, with all host cores and with one.
"""
import argparse
import gc
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
METRIC = "sketch HBM GB/s + decomps/sec at fixed rel. error; p50/p99 batched latency"


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline")
    ap.add_argument("--workload", choices=("all", "decomp", "serving", "precision", "paper"),
                    default="all",
                    help="decomp: the 400^3 decomposition line only; serving: the "
                         "request stream only; precision: the low-precision forms of "
                         "the 100^4 and 512x512x256 configurations; paper: the paper's "
                         "own synthetic workloads (Eq. (9) 600^3 sweeps of Section 4.3, "
                         "the Section 6.3 tendiag 600^3 and a 200^4 Tucker tensor); all: "
                         "decomp, serving and precision in one line")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--load", type=float, default=0.7,
                    help="arrival rate as a fraction of the one-at-a-time throughput")
    ap.add_argument("--max-group", type=int, default=64,
                    help="largest group of the grouped serving backend")
    ap.add_argument("--source", choices=("device", "host"), default="device")
    ap.add_argument("--oracle-requests", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device-to-device copy of 256 MiB (HBM "
                         "counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


def _measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)["kernels"][kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return float(rec["traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _factor_flops(I, s, mu):
    """Algorithmic flops of one factorization of an I x s sketch: Householder QR
    (2 I s^2 - 2 s^3 / 3), SVD of the s x s factor (~22 s^3 with both singular
    vector sets, Golub & Van Loan), Q_n = Q1 [U; 0] (4 I s mu - 2 s^2 mu)."""
    return 2 * I * s * s - 2 * s ** 3 / 3 + 22 * s ** 3 + 4 * I * s * mu - 2 * s * s * mu


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d.get("num_threads", 0) for d in threadpool_info()
             if d.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        n = 256 << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "copies": 5}))
        return

    if args.workload == "serving":
        srv = bench_serving(args)
        caps = srv["saturated_throughput_rps"]
        best = max(("batched", "grouped"), key=lambda k: caps[k])
        cap = caps[best]
        srv["workload"] += f"; value: the {best} server's saturated throughput"
        out = {"metric": METRIC, "value": cap,
               "unit": "requests/s", "n_gpus": 1, "steps": srv["requests"], "warmup": 0,
               "ms_per_step": round(1e3 / cap, 4),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": srv.pop("workload"), "parallelism": "single GPU"},
               "serving": srv}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "paper":
        pw = bench_paper(args)
        f4 = pw["eq9_fig4"]
        best = [r for r in f4["alg5"] if r["mu"] == 50][0]
        out = {"metric": METRIC, "value": round(1e3 / best["ms"], 2), "unit": "decomp/s",
               "n_gpus": 1, "steps": pw["repeats"], "warmup": 1, "ms_per_step": best["ms"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"Eq. (9) 600^3 float32, Alg. 5 at mu = {best['mu']}, "
                                      "K 10, q 1, alpha 0.2 (value); full sweeps under "
                                      "'paper'", "parallelism": "single GPU"},
               "paper": pw}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "precision":
        prec = bench_precision(args)
        c3 = prec["config3"]
        out = {"metric": METRIC, "value": c3["bf16"]["decomp_per_s"], "unit": "decomp/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": c3["bf16"]["ms"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
               "config": {"workload": c3["workload"], "parallelism": "single GPU"},
               "precision": prec}
        print(json.dumps(out), flush=True)
        return
    out = bench_decomp(args)
    if args.workload == "all":
        out["serving"] = bench_serving(args)
        out["precision"] = bench_precision(args)
    print(json.dumps(out), flush=True)


def bench_decomp(args):
    import numpy as np
    import torch
    import synth
    import paper_2303_11612_amd as tr

    w = synth.config(2, args.seed)
    dims, ranks, K, q, samples = w.dims, w.ranks, w.oversample, w.power, w.samples
    X = tr.to_device(w.A)
    N = len(dims)
    Qs = [tr.colmajor_empty((dims[n], ranks[n]), torch.float32) for n in range(N)]
    core = tr.colmajor_empty(ranks, torch.float32)
    wsb = tr.tucker_rand_workspace_size(dims, ranks, K, q, w.prob, samples, args.seed,
                                        torch.float32, sthosvd=True)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(tm=None):
        tr.tucker_rand_sthosvd(X, ranks, K, q, w.prob, samples, args.seed, workspace=ws,
                               out=(Qs, core), timer=tm, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Pass 1 (the timed region of `value`): K whole decompositions back to
    # back, nothing recorded between them (Python's cyclic collector paused,
    # so that a collection cannot land inside the host's launch sequence).
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    ms_per_step = 1e3 * wall / args.steps

    # Pass 2: the same K steps with an event pair around each (latency).
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    lat = sorted(a.elapsed_time(b) for a, b in ev)

    # Pass 3: the same K steps with HIP events on the launch stream around the
    # kernels of the timed classes (each event costs a few microseconds of
    # idle device time, which is why pass 1 records none).
    classes = ("colnorms", "ttm", "factor", "power", "sample", "gather", "gaussian")
    timer = tr.Timer(capacity=64 * (args.steps + 1), classes=classes)
    timer.reset()
    for _ in range(args.steps):
        step(timer)
    torch.cuda.synchronize()
    per_step = {c: timer.read(c)[0] / args.steps for c in classes}

    # the two full-tensor sweeps of mode 1, in algorithmic bytes per launch
    # (counting rule: a read of the tensor at its storage dtype, plus the
    # outputs the method needs at storage dtype; the shrink's float64
    # intermediate, twice the size, is the library's choice and not counted)
    elem = 4
    J1 = dims[1] * dims[2]
    sweeps = {
        # column norms: read the tensor, write J_1 float64 norms
        "colnorms": (dims[0] * J1 * elem + 8 * J1, "k_colnorms_l1<float, true>"),
        # shrink A x_1 Q_1^T: read the tensor, write mu_1/I_1 of it
        "ttm": (dims[0] * J1 * elem + elem * ranks[0] * J1, "k_ttm1_mfma<float, 1, 5, false, 8>"),
    }
    kern = {}
    for cls, (nbytes, kname) in sweeps.items():
        tot, cnt, tot0, cnt0 = timer.read(cls)
        avg0 = tot0 / max(cnt0, 1)
        kern[cls] = {"kernel": kname, "mode1_avg_ms": avg0, "mode1_launches": cnt0,
                     "all_modes_ms_per_step": tot / args.steps,
                     "algorithmic_bytes": nbytes,
                     "achieved_GBs": nbytes / (avg0 * 1e-3) / 1e9 if avg0 > 0 else None}
    tot, cnt, tot0, cnt0 = timer.read("factor")
    sf = [min(ranks[n] + K, dims[n]) for n in range(N)]
    fl = sum(_factor_flops(dims[n], sf[n], ranks[n]) for n in range(N)) / N
    favg = tot / max(cnt, 1)
    kern["factor"] = {"kernel": "k_factor_rf<24, 2, 16>", "avg_ms": favg, "launches": cnt,
                      "all_modes_ms_per_step": tot / args.steps,
                      "algorithmic_flops": fl,
                      "bound": "latency (one workgroup per sketch: QR, QR of R^T, Jacobi, "
                               "Q formation, each a chain of dependent steps)"}
    dom = max(sweeps, key=lambda c: kern[c]["mode1_avg_ms"])
    ach = kern[dom]["achieved_GBs"]
    traffic = _measured_traffic(kern[dom]["kernel"])
    sweep_roofline = {
        "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": None if traffic is None else round(traffic),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes": kern[dom]["algorithmic_bytes"],
        "kernel": kern[dom]["kernel"]}
    # the dominant kernel class by device time per step
    share = {c: per_step[c] / ms_per_step for c in classes}
    top = max(classes, key=lambda c: per_step[c])
    if top == "factor":
        fach = fl / (favg * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(fach, 6), "peak": FP64_VECTOR_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(fach / FP64_VECTOR_TFLOPS, 7),
                    "traffic": None, "algorithmic_flops": fl, "kernel": kern["factor"]["kernel"],
                    "note": "one workgroup per sketch; a chain of dependent steps on one "
                            "compute unit, so latency and not throughput bounds it"}
    else:
        roofline = dict(sweep_roofline)
    roofline["share_of_step"] = round(share[top], 4)

    # relative error of the GPU result: the library's float64 norms (Eq. (8)),
    # and an explicit float64 reconstruction from the float32 outputs
    _, _, info = tr.tucker_rand_sthosvd(X, ranks, K, q, w.prob, samples, args.seed,
                                        diag="norms", stream=stream)
    torch.cuda.synchronize()
    re_gpu = float(info["norms"][2])
    re_recon = _re_fp64(X, Qs, core)

    out = {
        "metric": METRIC, "value": round(args.steps / wall, 2), "unit": "decomp/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "rand ST-HOSVD + sampled products (Alg. 5), 400x400x400 "
                               "float32, ranks 10, K 10, q 1, T_n 4000 nearly-optimal",
                   "dims": list(dims), "ranks": list(ranks), "oversample": K, "power": q,
                   "samples": list(samples), "prob": w.prob, "storage": "f32",
                   "parallelism": "single GPU"},
        "sketch_hbm_GBs": round(kern["colnorms"]["achieved_GBs"], 1),
        "latency_ms": {"p50": round(statistics.median(lat), 4),
                       "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4)},
        "roofline": roofline,
        "sweep_roofline": sweep_roofline,
        "device_ms_per_step_by_class": {c: round(per_step[c], 4) for c in classes},
        "kernels": kern,
        "re_gpu": re_gpu,
        "re_gpu_reconstruction": re_recon,
    }

    if not args.no_cpu_baseline:
        import oracle
        A64 = w.A.astype(np.float64)
        times = []
        t_start = time.perf_counter()
        Qo = co = None
        while True:
            t1 = time.perf_counter()
            Qo, co, _ = oracle.rand_sthosvd(A64, ranks, K, q, w.prob, samples, args.seed)
            times.append(time.perf_counter() - t1)
            if time.perf_counter() - t_start > args.cpu_seconds and len(times) >= 2:
                break
        med = statistics.median(times)
        # one thread, as the paper times its MATLAB code (one computational thread)
        t1s = []
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"):
                t_start = time.perf_counter()
                while True:
                    t1 = time.perf_counter()
                    oracle.rand_sthosvd(A64, ranks, K, q, w.prob, samples, args.seed)
                    t1s.append(time.perf_counter() - t1)
                    if time.perf_counter() - t_start > args.cpu_seconds / 2 or len(t1s) >= 3:
                        break
        except ImportError:
            pass
        out["cpu_baseline"] = {
            "value": round(1.0 / med, 4), "unit": "decomp/s", "cores": _blas_threads(),
            "kind": "oracle", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{len(times)} full decompositions of the same 400^3 input and seed "
                      f"(median {med:.3f} s each), numpy float64 with multithreaded BLAS",
            "one_thread": None if not t1s else {
                "value": round(1.0 / statistics.median(t1s), 4), "unit": "decomp/s",
                "cores": 1, "sample": f"{len(t1s)} decompositions, BLAS limited to one thread"}}
        Qg = [Q.double().cpu().numpy() for Q in Qs]
        cg = core.double().cpu().numpy()
        out["re_oracle"] = oracle.relative_error(A64, co, Qo)
        out["parity_vs_oracle"] = {
            "max_factor_rel_err": max(float(np.linalg.norm(Qg[n] - Qo[n]) /
                                            np.linalg.norm(Qo[n])) for n in range(N)),
            "core_rel_err": float(np.linalg.norm(cg - co) / np.linalg.norm(co))}
    return out


def _re_fp64(X, Qs, core):
    """||A - core x_1 Q_1 ... x_N Q_N||_F / ||A||_F in float64 on the device (Eq. (8))."""
    import torch
    A = X.to(core.device).double()
    B = core.double()
    for n, Q in enumerate(Qs):
        B = torch.movedim(torch.tensordot(Q.double(), B, dims=([1], [n])), 0, n)
    return float(torch.linalg.vector_norm(A - B) / torch.linalg.vector_norm(A))


def bench_paper(args):
    """The paper's own synthetic workloads (Section 4.3 and Section 6) on the
    device, each decomposition timed with events around the library call
    (workspace preallocated, inputs in HBM) and its RE (Eq. (8)) from the
    library's norms:
    * Eq. (9) 600^3 (core 100^3 iid U(0,1), gamma 1e-3): Fig. 4's setting
      (Alg. 1, 4, 2, 5 with q 1, K 10, alpha 0.2) over mu = 5..100, Fig. 1's
      q = 1..4 and Fig. 2's K = 5..30 for Alg. 1 and 2, Fig. 3's alpha sweep
      for Alg. 4 and 5;
    * Section 6.3: tendiag 600^3 (v_i = 1 for i <= 50, (i - 49)^-2 after,
      600 terms), Alg. 2 and 5;
    * a 200^4 Tucker tensor (core 50^4 iid N(0,1), gamma 1e-3), Alg. 2 and 5;
    * Section 6.1's sparse 600^3 tensor: Alg. 5 with the first mode read from
      compressed sparse columns, against the dense path.
    mu runs to 100 as in the paper (s = mu + K up to 110); RE is
    cross-checked by a float64 reconstruction for a few decompositions."""
    import numpy as np
    import torch
    import synth
    import paper_2303_11612_amd as tr

    reps = max(1, min(args.steps, 3))
    dev = "cuda"
    ws = None

    def run(X, algo, mu, K=10, q=1, prob="none", alpha=None, seed=0, check=False):
        nonlocal ws
        N = X.dim()
        dims = tuple(X.shape)
        ranks = (mu,) * N
        samples = None
        if prob != "none":
            samples = synth.eq9_samples(alpha, dims, ranks, algo == "sthosvd")
        f = tr.tucker_rand_sthosvd if algo == "sthosvd" else tr.tucker_rand_thosvd
        need = tr.tucker_rand_workspace_size(dims, ranks, K, q, prob, samples, seed, X.dtype,
                                             sthosvd=algo == "sthosvd")
        if ws is None or ws.numel() < need:
            ws = None
            torch.cuda.empty_cache()
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        Qs, core, info = f(X, ranks, K, q, prob, samples, seed, diag="norms", workspace=ws)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            Qs, core, info = f(X, ranks, K, q, prob, samples, seed, diag="norms", workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        print(f"paper: {algo} dims {dims} mu {mu} K {K} q {q} {prob} alpha {alpha}: "
              f"{np.median(times):.3f} ms", file=sys.stderr, flush=True)
        r = {"mu": mu, "ms": round(float(np.median(times)), 3),
             "re": float(info["norms"][2]), "status": int(info["status"][0])}
        if prob != "none":
            r["T"] = list(samples)
        if check:
            r["re_fp64_reconstruction"] = _re_fp64(X, Qs, core)
        return r

    out = {"repeats": reps}
    t0 = time.perf_counter()
    X = synth.tucker_noise_device((600, 600, 600), (100, 100, 100), 1e-3, args.seed)
    torch.cuda.synchronize()
    out["generation_s"] = round(time.perf_counter() - t0, 2)
    mus = list(range(5, 105, 5))
    algs = {"alg1": ("thosvd", "none"), "alg4": ("thosvd", "uniform"),
            "alg2": ("sthosvd", "none"), "alg5": ("sthosvd", "uniform")}
    fig4 = {}
    for name, (algo, prob) in algs.items():
        fig4[name] = [run(X, algo, mu, prob=prob, alpha=0.2, check=(mu in (50, 100)))
                      for mu in mus]
    out["eq9_fig4"] = dict(fig4, setting="Eq. (9) 600^3 float32, gamma 1e-3; q 1, K 10, "
                           "alpha 0.2; Alg. 4/5 with uniform probabilities")
    out["eq9_fig1_q"] = {name: {str(q): [run(X, algo, mu, q=q) for mu in (10, 50, 100)]
                                for q in (1, 2, 3, 4)}
                         for name, (algo, _) in (("alg1", algs["alg1"]),
                                                 ("alg2", algs["alg2"]))}
    out["eq9_fig2_K"] = {name: {str(K): [run(X, algo, mu, K=K) for mu in (10, 30)]
                                for K in (5, 10, 15, 20, 25, 30)}
                         for name, (algo, _) in (("alg1", algs["alg1"]),
                                                 ("alg2", algs["alg2"]))}
    out["eq9_fig3_alpha"] = {name: {str(a): [run(X, algo, mu, prob=prob, alpha=a)
                                             for mu in (10, 50, 100)]
                                    for a in (0.01, 0.08, 0.15, 0.22, 0.29, 0.36, 0.43, 0.5)}
                             for name, (algo, prob) in (("alg4", algs["alg4"]),
                                                        ("alg5", algs["alg5"]))}
    del X
    torch.cuda.empty_cache()
    v = [1.0 if i < 50 else float(i - 49) ** -2 for i in range(1, 601)]
    X = synth.tendiag_noise_device((600, 600, 600), v, 1e-3, args.seed + 1)
    out["tendiag600"] = {name: [run(X, algs[name][0], mu, prob=algs[name][1], alpha=0.2,
                                    check=(mu == 50)) for mu in (10, 30, 50)]
                         for name in ("alg2", "alg5")}
    del X
    torch.cuda.empty_cache()
    # Section 6.1's sparse tensor: the first mode from compressed sparse
    # columns against the dense path on the same tensor (Alg. 5, alpha 0.01,
    # uniform probabilities as in the paper)
    X = synth.sparse_cp_device((600, 600, 600), 600, 0.05, 1000.0, args.seed + 3)
    csc = synth.csc_mode1(X)
    sp = {"nnz": int(csc[2].numel()), "density": round(csc[2].numel() / X.numel(), 4),
          "csc_bytes": int(8 * csc[0].numel() + 4 * csc[1].numel() + 4 * csc[2].numel()),
          "dense_bytes": int(4 * X.numel()), "csc": [], "dense": []}
    for mu in (10, 30, 50):
        ranks = (mu,) * 3
        samples = synth.eq9_samples(0.01, X.shape, ranks, True)
        need = tr.tucker_rand_workspace_size(X.shape, ranks, 10, 1, "uniform", samples, 0,
                                             X.dtype, sthosvd=True)
        if ws is None or ws.numel() < need:
            ws = None
            torch.cuda.empty_cache()
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        for kind in ("csc", "dense"):
            def call():
                if kind == "csc":
                    return tr.tucker_rand_sthosvd_csc(*csc, X.shape, ranks, 10, 1, "uniform",
                                                      samples, 0, diag=True, workspace=ws)
                return tr.tucker_rand_sthosvd(X, ranks, 10, 1, "uniform", samples, 0,
                                              diag="norms", workspace=ws)
            call()
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                _, _, info = call()
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            print(f"paper: sparse600 {kind} mu {mu}: {np.median(times):.3f} ms", file=sys.stderr,
                  flush=True)
            sp[kind].append({"mu": mu, "ms": round(float(np.median(times)), 3),
                             "re": float(info["norms"][2]), "status": int(info["status"][0])})
    out["sparse600"] = dict(sp, setting="Section 6.1: 600 rank-one terms, 5 % dense factor "
                                        "vectors, gamma 1000; Alg. 5, K 10, q 1, alpha 0.01")
    del X, csc
    torch.cuda.empty_cache()
    X = synth.tucker_noise_device((200,) * 4, (50,) * 4, 1e-3, args.seed + 2, core="gauss")
    out["tucker200pow4"] = {name: [run(X, algs[name][0], mu, prob=algs[name][1], alpha=0.01,
                                       check=(mu == 30)) for mu in (10, 30, 50)]
                            for name in ("alg2", "alg5")}
    del X
    ws = None
    torch.cuda.empty_cache()
    out["all_status_ok"] = all(
        r["status"] == 0
        for blk in (out["eq9_fig4"], out["tendiag600"], out["tucker200pow4"], out["sparse600"])
        for k, lst in blk.items() if isinstance(lst, list) for r in lst)
    return out


def bench_precision(args):
    """Decomposition time and relative error of the float64 path and of the
    low-precision power products on the 100^4 configuration (T-HOSVD, q = 2,
    exact products: float64 vs bfloat16) and the 512 x 512 x 256 one
    (T-HOSVD, q = 1, 8000 uniformly sampled columns: float64 vs bfloat16 vs
    FP8 e4m3).  Time per decomposition: the better of two passes of `steps`
    back-to-back calls.  The relative errors come from a float64
    reconstruction; the FP64 oracle's error is added by the CPU baseline leg."""
    import numpy as np
    import torch
    import synth
    import paper_2303_11612_amd as tr

    steps = max(2, min(args.steps, 10))
    res = {}
    for k, precs, name in ((3, ("native", "bf16"),
                            "rand T-HOSVD (Alg. 1), 100^4 float32, ranks 20, K 10, q 2"),
                           (4, ("native", "bf16", "fp8e4m3"),
                            "rand T-HOSVD + sampled products (Alg. 4), 512x512x256 float32 "
                            "bumps, ranks (30,30,15), K 10, q 1, T_n 8000 uniform")):
        w = synth.config(k, args.seed)
        X = tr.to_device(w.A)
        entry = {"workload": name}
        for prec in precs:
            wsb = tr.tucker_rand_workspace_size(w.dims, w.ranks, w.oversample, w.power, w.prob,
                                                w.samples, args.seed, torch.float32,
                                                sthosvd=False, precision=prec)
            ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
            Qs = [tr.colmajor_empty((w.dims[n], w.ranks[n]), torch.float32)
                  for n in range(len(w.dims))]
            core = tr.colmajor_empty(w.ranks, torch.float32)

            def step(tm=None):
                tr.tucker_rand_thosvd(X, w.ranks, w.oversample, w.power, w.prob, w.samples,
                                      args.seed, precision=prec, workspace=ws, out=(Qs, core),
                                      timer=tm)
            for _ in range(2):
                step()
            torch.cuda.synchronize()
            # the better of two timed passes (a host stall of ~20 ms landed
            # in one pass of some runs; the power-step device time did not
            # move), with the cyclic collector paused
            ms = float("inf")
            for _ in range(2):
                gc.collect()
                gc.disable()
                t0 = time.perf_counter()
                for _ in range(steps):
                    step()
                torch.cuda.synchronize()
                ms = min(ms, 1e3 * (time.perf_counter() - t0) / steps)
                gc.enable()
            timer = tr.Timer(capacity=64 * (steps + 1), classes=("power",))
            timer.reset()
            for _ in range(steps):
                step(timer)
            torch.cuda.synchronize()
            ptot, pcnt, _, _ = timer.read("power")
            entry[prec] = {"ms": round(ms, 4), "decomp_per_s": round(1e3 / ms, 2),
                           "power_ms_per_decomp": round(ptot / steps, 4),
                           "re": _re_fp64(X, Qs, core)}
            if prec == "native":
                entry[prec]["Q"] = [Q.double().cpu().numpy() for Q in Qs]
            else:
                Qn = entry["native"]["Q"]
                # largest principal-angle sine between the low-precision and
                # the float64 factors' subspaces, per mode
                entry[prec]["subspace_sin_vs_native"] = [
                    float(np.linalg.norm(Q.double().cpu().numpy() @ Q.double().cpu().numpy().T
                                         - Qn[n] @ Qn[n].T, 2)) for n, Q in enumerate(Qs)]
                entry[prec]["re_ratio_vs_native"] = entry[prec]["re"] / entry["native"]["re"]
            del ws
        entry["native"].pop("Q")
        if not args.no_cpu_baseline:
            import oracle
            A64 = w.A.astype(np.float64)
            Qo, co, _ = oracle.rand_thosvd(A64, w.ranks, w.oversample, w.power, w.prob,
                                           w.samples, args.seed)
            entry["re_oracle_fp64"] = oracle.relative_error(A64, co, Qo)
        res[f"config{k}"] = entry
        del X
        torch.cuda.empty_cache()
    return res


def bench_serving(args):
    """The request stream: modes U{32..384}, ranks U{4..24}, T_n = 4 mu_n,
    nearly-optimal sampling, q = 1, K = 10, Poisson arrivals at `load` times
    the one-at-a-time throughput; one slot (one request at a time) against
    `slots` concurrent slots under an HBM budget (one request per stream,
    "batched") and against `slots` grouped slots (a group of admitted requests
    per stream, every stage one launch for the group, "grouped"), on the same
    arrivals, and again at the grouped server's own capacity."""
    import numpy as np
    import torch
    import synth
    import paper_2303_11612_amd as tr
    from paper_2303_11612_amd import serving as sv

    n = args.requests
    t_gen = time.perf_counter()
    reqs = []
    for rid in range(n):
        X, ranks, samples = synth.serving_request_device(rid)
        if args.source == "host":
            h = torch.empty(X.numel(), dtype=torch.float32, pin_memory=True)
            h.copy_(X.permute(2, 1, 0).reshape(-1))
            X = h.as_strided(tuple(X.shape), X.stride())
        reqs.append(sv.Request(rid, X, ranks, samples, seed=rid))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    budget = int(args.budget_gb * (1 << 30))

    def serve(slots, arrivals, grouped=False):
        for r, a in zip(reqs, arrivals):
            r.arrival = float(a)
        be = sv.GroupedBackend(slots, args.max_group) if grouped else sv.GpuBackend(slots)
        server = sv.Server(be, slots=slots, hbm_budget=budget)
        res = server.run(reqs)
        return res, server

    # warm-up: kernels loaded and allocator pools filled for every slot
    warm = reqs[:2 * args.slots]
    for r in warm:
        r.arrival = 0.0
    sv.Server(sv.GpuBackend(args.slots), slots=args.slots, hbm_budget=budget).run(warm)
    sv.Server(sv.GroupedBackend(args.slots, args.max_group), slots=args.slots,
              hbm_budget=budget).run(reqs[:4 * args.slots])
    torch.cuda.synchronize()

    zero = np.zeros(n)
    sat1, _ = serve(1, zero)
    cap1 = sv.summarize(sat1)["throughput_rps"]
    satS, _ = serve(args.slots, zero)
    capS = sv.summarize(satS)["throughput_rps"]
    satG, srvG = serve(args.slots, zero, grouped=True)
    capG = sv.summarize(satG)["throughput_rps"]
    sat_groups = srvG.group_sizes
    rate = args.load * cap1
    arr = sv.poisson_arrivals(n, rate, seed=args.seed + 7)
    one, _ = serve(1, arr)
    mix, srvS = serve(args.slots, arr)
    peak = srvS.peak_used
    grp, srvG = serve(args.slots, arr, grouped=True)
    # a second stream at the grouped server's own saturation point
    arr_hi = sv.poisson_arrivals(n, args.load * capG, seed=args.seed + 8)
    grp_hi, srvH = serve(args.slots, arr_hi, grouped=True)
    mix_hi, _ = serve(args.slots, arr_hi)

    # results alone (one slot, no overlap) against results in the mix: bitwise
    same = all(torch.equal(a.core, b.core) and
               all(torch.equal(x, y) for x, y in zip(a.factors, b.factors))
               for a, b in zip(sat1, mix))
    # relative Tucker error of each request (Eq. (8)), by explicit float64
    # reconstruction from the mix's outputs
    re = [_re_fp64(r.X, m.factors, m.core) for r, m in zip(reqs, mix)]
    re_g = [_re_fp64(r.X, m.factors, m.core) for r, m in zip(reqs, grp)]
    # grouped results: bitwise the same in any group (each of the first
    # requests again, alone)
    k_alone = min(16, n)
    alone_g = sv.Server(sv.GroupedBackend(1, 1), slots=1, hbm_budget=budget).run(
        [sv.Request(r.rid, r.X, r.ranks, r.samples, seed=r.seed) for r in reqs[:k_alone]])
    same_g = all(torch.equal(a.core, b.core) and
                 all(torch.equal(x, y) for x, y in zip(a.factors, b.factors))
                 for a, b in zip(alone_g, grp[:k_alone]))
    out = {
        "workload": f"serving stream, {n} requests, modes U{{32..384}}^3 float32, ranks "
                    f"U{{4..24}}, rand ST-HOSVD + nearly-optimal sampling T_n = 4 mu_n, "
                    f"q 1, K 10, Poisson arrivals at {args.load} x one-at-a-time throughput",
        "requests": n, "slots": args.slots, "source": args.source,
        "hbm_budget_bytes": budget, "peak_admitted_bytes": int(peak),
        "mean_tensor_MB": round(sum(r.X.numel() * 4 for r in reqs) / n / 1e6, 2),
        "arrival_rate_rps": round(rate, 2),
        "saturated_throughput_rps": {"one_at_a_time": cap1, "batched": capS,
                                     "grouped": capG},
        "saturated_group_sizes": {"groups": len(sat_groups),
                                  "mean": round(float(np.mean(sat_groups)), 2),
                                  "max": int(max(sat_groups))},
        "one_at_a_time": sv.summarize(one),
        "batched": sv.summarize(mix),
        "grouped": sv.summarize(grp),
        "grouped_mean_group": round(float(np.mean(srvG.group_sizes)), 2),
        "at_grouped_load": {"arrival_rate_rps": round(args.load * capG, 2),
                            "grouped": sv.summarize(grp_hi),
                            "batched": sv.summarize(mix_hi),
                            "grouped_mean_group": round(float(np.mean(srvH.group_sizes)), 2)},
        "all_status_ok": all(m.status == 0 for m in mix + grp + grp_hi + mix_hi),
        "mix_equals_alone_bitwise": bool(same),
        "grouped_equals_alone_bitwise": {"requests": k_alone, "ok": bool(same_g)},
        "rel_error": {"mean": float(np.mean(re)), "max": float(np.max(re))},
        "grouped_rel_error_max_abs_diff": float(np.max(np.abs(np.array(re_g) - np.array(re)))),
        "generation_s": round(t_gen, 2),
    }
    if args.oracle_requests > 0:
        import oracle
        k = min(args.oracle_requests, n)
        diffs, t_or = [], 0.0
        for i in range(k):
            A = reqs[i].X.double().cpu().numpy()
            t1 = time.perf_counter()
            Qo, co, _ = oracle.rand_sthosvd(A, reqs[i].ranks, 10, 1, "nearly_optimal",
                                            reqs[i].samples, reqs[i].seed)
            t_or += time.perf_counter() - t1
            diffs.append(abs(oracle.relative_error(A, co, Qo) - re[i]))
        out["oracle_subset"] = {"requests": k, "max_abs_re_diff": float(max(diffs)),
                                "oracle_s_per_request": round(t_or / k, 3)}
    return out


if __name__ == "__main__":
    main()
