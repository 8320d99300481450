"""Benchmark: n = 16384 partial symmetric eigensolve (QDWHpartial-EIG, FP64) on one MI355X.

Workload (default): A = Q diag(lambda) Q^T, n = 16384, Q Haar, 90% of the
eigenvalues uniform on [-1, 0.5] and 10% in 8 clusters of width 1e-8 in
[0.5, 1]; the top 20% (3277) eigenpairs are wanted.  One step = one full
solve (estimator, three DWH steps, projector QR, Rayleigh-Ritz) with A
already resident in HBM.

Prints one JSON line.  Besides the time to solution it reports
  * roofline: the FP64 MFMA GEMM kernel (the dominant kernel), algorithmic
    flops / summed kernel time from hipEvents around each of its launches
    during the timed steps, against the 78.6 TFLOP/s FP64 peak;
  * cpu_baseline: the CPU oracle timed on a bounded sample of the same
    workload (smaller n, same spectrum recipe), scaled to n = 16384 by n^3.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
METRIC = "n=16K partial EIG/SVD time-to-solve, MFMA %peak; served solves/s + p50/p99"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--fraction", type=float, default=0.2)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work to aim for")
    p.add_argument("--no-serve", action="store_true", help="skip the batched and served request-mix legs")
    p.add_argument("--gemm-probe", action="store_true",
                   help="only the 1 GiB copy and the two dominant n^3 GEMM shapes of a Cholesky step "
                        "(for HBM byte counters), then exit")
    p.add_argument("--copy-probe", action="store_true",
                   help="first copy 1 GiB device to device (calibrates HBM byte counters under rocprofv3 --pmc)")
    p.add_argument("--serve-requests", type=int, default=48)
    p.add_argument("--serve-rate", type=float, default=3.0, help="Poisson arrival rate (requests/s)")
    return p.parse_args()


def build_mix(torch, trace):
    """Device matrices for a request trace (planted spectra, built before timing)."""
    from synthetic import eig_uniform, svd_geometric
    import numpy as np
    dev = torch.device("cuda")
    out = []
    for r in trace:
        if r["kind"] == "eig":
            A, lam = eig_uniform(r["n"], r["seed"], device=dev)
            out.append((dict(type="eig", A=A, fraction=r["fraction"]), np.sort(lam)[::-1]))
        else:
            A, sig = svd_geometric(r["n"], r["n"], r["seed"], kappa=r["kappa"], device=dev)
            out.append((dict(type="svd", A=A, k=r["k"]), np.asarray(sig)))
    return out


def _vals(spec, res):
    return (res[0] if spec["type"] == "eig" else res[1]).cpu().numpy()


def _relerr(spec, res, exact):
    import numpy as np
    v = _vals(spec, res)
    e = exact[:len(v)]
    return float(np.max(np.abs(v - e) / np.abs(e)))


def batched_leg(q, torch, mix):
    """The same ragged batch solved one call at a time and with qdwhp_batched."""
    specs = [m[0] for m in mix]
    for sp in specs[:2]:
        (q.eig(sp["A"], fraction=sp["fraction"]) if sp["type"] == "eig" else q.svd(sp["A"], sp["k"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [(q.eig(sp["A"], fraction=sp["fraction"]) if sp["type"] == "eig" else q.svd(sp["A"], sp["k"]))
           for sp in specs]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    q.batched(specs[:4])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = q.batched(specs)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    same = all(all(bool((x == y).all()) for x, y in zip(a, b)) for a, b in zip(seq, res))
    err = max(_relerr(sp, r, m[1]) for sp, r, m in zip(specs, res, mix))
    return {"problems": len(specs), "sequential_s": t_seq, "batched_s": t_bat,
            "sequential_solves_per_s": len(specs) / t_seq, "batched_solves_per_s": len(specs) / t_bat,
            "speedup": t_seq / t_bat, "lanes": q.tune_get("batch.lanes", 8),
            "bitwise_equal_to_standalone": same, "max_rel_value_err": err}


def serve_leg(q, torch, mix, trace, precision):
    """Open-loop Poisson arrivals into the request server; latency = arrival to results ready."""
    import numpy as np
    opts = q.default_opts(precision=precision)
    lat, qms, errs, done_t = [], [], [], []
    with q.Server(arena_bytes=64 << 30, lanes=0, opts=opts) as srv:
        warm = srv.submit(mix[0][0])
        srv.poll(warm)
        t0 = time.perf_counter()
        tickets = []
        for (spec, exact), r in zip(mix, trace):
            delay = r["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(spec))
        failed = []
        for i, ((spec, exact), tk) in enumerate(zip(mix, tickets)):
            try:
                res, info, l, qm = srv.poll(tk)
            except q.QdwhpError as e:
                failed.append((i, e.status))
                continue
            lat.append(l); qms.append(qm)
            done_t.append(time.perf_counter() - t0)
            errs.append(_relerr(spec, res, exact))
        span = time.perf_counter() - t0
    lat = np.array(lat)
    return {"precision": "fp64" if precision == 0 else "mixed_fp32", "requests": len(lat),
            "offered_rate_per_s": len(trace) / trace[-1]["arrival"],
            "solves_per_s": len(lat) / span, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_queue_ms": float(np.mean(qms)),
            "max_rel_value_err": float(max(errs)), "failed": failed}


def cpu_baseline(n_full, fraction, budget):
    """Time the oracle on the same workload recipe at a reduced size."""
    import oracle
    from synthetic import eig_clustered
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    ns = 512
    t = 0.0
    while True:
        A, lam = eig_clustered(ns, 1002)
        t0 = time.perf_counter()
        r = oracle.eig_partial(A, fraction=fraction)
        t = time.perf_counter() - t0
        # next size costs ~8x: stop when that would exceed the budget
        if t * 8.0 > budget or 2 * ns > n_full:
            break
        ns *= 2
    exact = np.sort(lam)[::-1][:r["k"]]
    err = float(np.max(np.abs(r["w"] - exact) / np.abs(exact)))
    scaled = t * (n_full / ns) ** 3
    return dict(value=scaled, unit="s", cores=int(threads), kind="oracle",
                sample=f"oracle eig_partial on the same spectrum recipe at n={ns} "
                       f"(top {fraction:.0%}) took {t:.2f} s; scaled by (n/{ns})^3 to n={n_full}; "
                       f"max rel value err {err:.1e}")


def gemm_probe(torch, dev, n):
    """Copy calibration (1 GiB read + written, twice), the dominant GEMMs of
    a Cholesky-based step at size n: Z = X^T X (upper tiles) and X W (full),
    in FP64 and with FP32 operands (twice each), and a Householder QR of an
    n x n/8 matrix (the panel kernels of the projector and stacked QRs)."""
    import ctypes
    import paper_2104_14186_amd as q
    x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    x.fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    del x, y
    X = torch.empty((n, n), dtype=torch.float64, device=dev)
    W = torch.empty((n, n), dtype=torch.float64, device=dev)
    Z = torch.empty((n, n), dtype=torch.float64, device=dev)
    X.fill_(1.0 / n)
    W.fill_(1.0 / n)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = q.lib()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    for f32 in (0, 2):
        for _ in range(2):
            assert L.qdwhp_dgemm(1, 0, n, n, n, 1.0, p(X), n, p(X), n, 0.0, p(Z), n, 1 | f32, st) == 0
            assert L.qdwhp_dgemm(0, 0, n, n, n, 1.0, p(X), n, p(W), n, 0.0, p(Z), n, f32, st) == 0
    torch.cuda.synchronize()
    del W, Z
    nc = max(1, n // 8)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    P = torch.randn((nc, n), dtype=torch.float64, device=dev, generator=g)   # column-major n x nc
    tau = torch.empty(nc, dtype=torch.float64, device=dev)
    nbytes = L.qdwhp_geqrf_workspace(n, nc)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    assert L.qdwhp_geqrf(p(P), n, nc, n, p(tau), p(ws), nbytes, st) == 0
    torch.cuda.synchronize()
    print(json.dumps({"gemm_probe": n, "qr_probe": [n, nc]}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2104_14186_amd as q
    from synthetic import eig_clustered

    dev = torch.device("cuda:0")
    if args.gemm_probe:
        gemm_probe(torch, dev, args.n)
        return
    if args.copy_probe:
        x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        x.fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)                       # 1 GiB read + 1 GiB written
        torch.mul(x, 2.0, out=y)         # the same through an elementwise kernel
        torch.cuda.synchronize()
        del x, y
    n, f = args.n, args.fraction
    print(f"[bench] generating n={n} planted matrix", file=sys.stderr, flush=True)
    A, lam = eig_clustered(n, 1002, device=dev)
    A = A.contiguous()              # symmetric: row-major storage is the column-major matrix
    torch.cuda.synchronize()
    k = min(n, max(1, int(math.floor(f * n + 0.5))))
    opts = q.default_opts()
    lib = q.lib()
    import ctypes
    nbytes = lib.qdwhp_eig_workspace(n, f, ctypes.byref(opts))
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    w = torch.empty(k, dtype=torch.float64, device=dev)
    Vb = torch.empty((k, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    info = q.Info()

    def solve():
        st = lib.qdwhp_eig(ctypes.c_void_p(A.data_ptr()), n, n, f, q.LARGEST,
                           ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(Vb.data_ptr()), n,
                           ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.byref(opts),
                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(info))
        if st != 0:
            raise RuntimeError(f"qdwhp_eig failed with status {st}")

    for i in range(args.warmup):
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
        solve()
    torch.cuda.synchronize()
    q.profile_begin()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for i in range(args.steps):
        solve()
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gflops, gms, glaunch = q.profile_end()
    ms_step = e0.elapsed_time(e1) / args.steps
    d = info.as_dict()

    # accuracy of the last solve against the planted spectrum, and sampled residuals
    exact = np.sort(lam)[::-1][:k]
    wv = w.cpu().numpy()
    rel = float(np.max(np.abs(wv - exact) / np.abs(exact)))
    cols = torch.linspace(0, k - 1, 8, device=dev).long()
    Vs = Vb[cols].t().contiguous()               # n x 8 sampled eigenvectors
    R = A @ Vs - Vs * w[cols][None, :]
    resid = float((R.norm(dim=0) / float(np.max(np.abs(lam)))).max())

    achieved = gflops / (gms * 1e-3) / 1e12 if gms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": ms_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"eig{n}_top{int(round(100 * f))}pct_clustered", "n": n, "k": k,
                   "fraction": f, "spectrum": "90% U[-1,0.5] + 8 clusters width 1e-8 in [0.5,1]",
                   "seed": 1002, "parallelism": "single_gpu"},
        "solves_per_s": 1e3 / ms_step,
        "mfma_frac_table1": d["flops_table1"] / (ms_step * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
        "phases_ms": dict(zip(["estimator", "iterations", "projector_qr", "q2", "rr_products",
                               "small_solve", "vectors", "total"], [round(x, 2) for x in d["ms"]])),
        "solver": {kk: d[kk] for kk in ["ell", "ind", "kinds", "jacobi_sweeps", "rr_split", "tau", "retries"]},
        "accuracy": {"max_rel_value_err": rel, "sampled_residual": resid},
        "roofline": {"bound": "mfma", "kernel": "dgemm_kernel (FP64 v_mfma_f64_16x16x4f64)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "launches": glaunch, "kernel_ms_per_step": gms / args.steps,
                     "algorithmic_flops_per_launch": gflops / max(glaunch, 1)},
    }
    if not args.no_serve:
        from synthetic import request_trace, CONFIG_SEEDS
        trace = request_trace(args.serve_requests, args.serve_rate, CONFIG_SEEDS["trace"])
        print("[bench] building request mix", file=sys.stderr, flush=True)
        mix = build_mix(torch, trace)
        print("[bench] batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(q, torch, mix[:24])
        print("[bench] served leg fp64", file=sys.stderr, flush=True)
        out["serving"] = serve_leg(q, torch, mix, trace, q.FP64)
        print("[bench] served leg mixed", file=sys.stderr, flush=True)
        out["serving_mixed"] = serve_leg(q, torch, mix, trace, q.MIXED_FP32)
        out["serving"]["trace"] = (f"{len(trace)} requests, Poisson {args.serve_rate}/s, 60% EIG / 40% SVD, "
                                   "n in {256..4096}, fraction U[1%,20%], SVD kappa 10^U[0,12]")
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, f, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
