"""Benchmark: n = 16384 partial symmetric eigensolve (QDWHpartial-EIG, FP64) on one MI355X.

Workload (headline): A = Q diag(lambda) Q^T, n = 16384, Q Haar, 90% of the
eigenvalues uniform on [-1, 0.5] and 10% in 8 clusters of width 1e-8 in
[0.5, 1]; the top 20% (3277) eigenpairs are wanted.  One step = one full
solve (estimator, three DWH steps, projector QR, Rayleigh-Ritz) with A
already resident in HBM; the timed steps run without any profiling hooks.

Prints one JSON line.  Besides the time to solution it reports
  * roofline: the FP64 MFMA GEMM kernel (the dominant kernel): algorithmic
    flops / summed kernel time from hipEvents around each of its launches
    during one extra solve after the timed ones, against the 78.6 TFLOP/s
    FP64 peak; traffic = HBM bytes per launch from the committed
    rocprofv3 counter summary when it was taken on the current GEMM source;
  * workloads: the other benchmark configurations (n = 16384 top 1%, the
    4096^2 kappa = 1e16 SVD, the 16384 x 8192 SVD in FP64 and mixed
    precision, n = 512), each with time, Table 1 flop rate, value error
    against the planted spectrum and the residual over all returned vectors;
  * batched / serving: a ragged request mix (batched vs one call at a time;
    closed-loop capacity of the server, then an open-loop Poisson trace at
    0.7x that capacity, FP64 and mixed);
  * cpu_baseline: the CPU oracle timed on the same spectrum recipe at
    n = 4096 and, when the budget allows, 8192, scaled to n = 16384 by n^3.
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
    p.add_argument("--cpu-budget", type=float, default=150.0,
                   help="the oracle also runs at n = 8192 when 8x its n = 4096 time fits this (s)")
    p.add_argument("--no-workloads", action="store_true", help="skip the other benchmark configurations")
    p.add_argument("--no-roofline", action="store_true",
                   help="skip the extra solve with per-launch GEMM events (for counter runs under rocprofv3)")
    p.add_argument("--input", default="", help="load the headline matrix (and *_lam.npy) from this .npy "
                   "instead of generating it on the device")
    p.add_argument("--write-input", default="", help="write the generated headline matrix to this .npy and exit")
    p.add_argument("--no-serve", action="store_true", help="skip the batched and served request-mix legs")
    p.add_argument("--gemm-probe", action="store_true",
                   help="only the 1 GiB copy and the two dominant n^3 GEMM shapes of a Cholesky step "
                        "(for HBM byte counters), then exit")
    p.add_argument("--copy-probe", action="store_true",
                   help="first copy 1 GiB device to device (calibrates HBM byte counters under rocprofv3 --pmc)")
    p.add_argument("--serve-requests", type=int, default=48)
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


def same_shape_leg(q, torch, n=1024, count=16):
    """count EIG problems of one size n (top 10%, uniform planted spectra):
    one call at a time, batched with grouped iterations, and batched with
    every instance on its own lane (batch.grouped = 0)."""
    from synthetic import eig_uniform
    dev = torch.device("cuda")
    specs = [dict(type="eig", A=eig_uniform(n, 42000 + i, device=dev)[0], fraction=0.1) for i in range(count)]
    q.batched(specs[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [q.eig(sp["A"], fraction=sp["fraction"]) for sp in specs]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {"problems": count, "n": n, "sequential_s": t_seq}
    for grouped in (1, 0):
        q.tune_set("batch.grouped", grouped)
        q.batched(specs[:2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = q.batched(specs)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        same = all(all(bool((x == y).all()) for x, y in zip(a, b)) for a, b in zip(seq, res))
        key = "grouped" if grouped else "per_lane"
        out[key] = {"s": t, "solves_per_s": count / t, "speedup_vs_sequential": t_seq / t,
                    "bitwise_equal_to_standalone": same}
    q.tune_set("batch.grouped", 1)
    return out


def serve_leg(q, torch, mix, trace, precision):
    """The request server, first closed loop (every request submitted at
    once, so the lanes never idle: capacity = requests / span), then the
    trace's Poisson arrivals replayed open loop at 0.7x that capacity;
    latency = submit to results ready.  Reports throughput, p50/p99 latency,
    the arena high-water mark and the value error against the planted spectra."""
    opts = q.default_opts(precision=precision)
    out = {"precision": "fp64" if precision == 0 else "mixed_fp32", "requests": len(mix)}
    with q.Server(arena_bytes=64 << 30, lanes=0, opts=opts) as srv:
        warm = srv.submit(mix[0][0])
        srv.poll(warm)
        srv.stats(reset=True)
        t0 = time.perf_counter()
        tickets = [srv.submit(spec) for spec, _ in mix]
        for tk in tickets:
            srv.poll(tk)
        span = time.perf_counter() - t0
        cap = len(mix) / span
        st = srv.stats(reset=True)
        out["closed_loop"] = {"solves_per_s": cap, "span_s": span, "arena_peak_bytes": st["arena_peak_bytes"],
                              "peak_running": st["peak_running"], "iteration_groups": st["groups"],
                              "grouped_requests": st["grouped_requests"]}
        rate = 0.7 * cap
        lat, qms, errs = [], [], []
        t0 = time.perf_counter()
        tickets = []
        for (spec, exact), r in zip(mix, trace):
            delay = r["arrival"] / rate - (time.perf_counter() - t0)   # trace drawn at rate 1
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
            lat.append(l)
            qms.append(qm)
            errs.append(_relerr(spec, res, exact))
        span = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array(lat)
    out["open_loop"] = {"offered_rate_per_s": rate, "solves_per_s": len(lat) / span,
                        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "max_ms": float(lat.max()), "mean_queue_ms": float(np.mean(qms)),
                        "arena_peak_bytes": st["arena_peak_bytes"], "arena_bytes": st["arena_bytes"],
                        "peak_running": st["peak_running"], "iteration_groups": st["groups"],
                        "grouped_requests": st["grouped_requests"],
                        "max_rel_value_err": float(max(errs)), "failed": failed}
    out["trace"] = (f"{len(mix)} requests, Poisson arrivals at 0.7x the closed-loop capacity, 60% EIG / 40% SVD, "
                    "n in {256..4096}, fraction U[1%,20%], SVD kappa 10^U[0,12]")
    return out


def _host_info():
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return cpu, nproc


def cpu_baseline(n_full, fraction, budget):
    """Time the oracle on the same workload recipe (same tol as the library)
    at n = 4096 and, when the n^3 extrapolation of that run fits the budget,
    at 8192; the largest run is scaled to n_full by n^3."""
    import oracle
    from synthetic import eig_clustered
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    cpu, nproc = _host_info()
    runs = {}
    ns = 4096
    while True:
        A, lam = eig_clustered(ns, 1002)
        t0 = time.perf_counter()
        r = oracle.eig_partial(A, fraction=fraction, tol=0.05)
        t = time.perf_counter() - t0
        exact = np.sort(lam)[::-1][:r["k"]]
        runs[ns] = (t, float(np.max(np.abs(r["w"] - exact) / np.abs(exact))))
        print(f"[bench] oracle n={ns}: {t:.1f} s", file=sys.stderr, flush=True)
        if 2 * ns > n_full or t * 8.0 > budget:
            break
        ns *= 2
    t, err = runs[ns]
    return dict(value=t * (n_full / ns) ** 3, unit="s", cores=int(threads), kind="oracle",
                host_cpu=cpu, host_nproc=nproc,
                runs_s={str(k): round(v[0], 2) for k, v in runs.items()},
                sample=f"oracle eig_partial (NumPy/SciPy FP64, {threads} BLAS threads on {nproc} host CPUs) "
                       f"on the same spectrum recipe at n={ns} (top {fraction:.0%}) took {t:.2f} s; "
                       f"scaled by (n/{ns})^3 to n={n_full} (a factor {(n_full / ns) ** 3:.0f}); "
                       f"max rel value err {err:.1e}")


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "dgemm_kernel_eig16384_top20_traffic.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2104_14186_amd", "csrc", "gemm.hip")


def traffic_from_profile():
    """HBM bytes per dgemm_kernel launch from the committed counter summary,
    or None when it is missing or was taken on another version of the GEMM
    source (sha256 recorded in the summary)."""
    import hashlib
    try:
        text = open(TRAFFIC_SUMMARY).read()
        sha = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            key, _, v = line[2:].partition(":")
            vals[key.strip()] = v.strip().strip("`")
    if vals.get("gemm.hip sha256") != sha:
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def _time_calls(torch, fn, warmup, steps):
    """Median and all per-call times (ms) from torch events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    stream = torch.cuda.current_stream()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), ts


def eig_entry(q, torch, name, A, lam, f, opts=None, warmup=1, steps=2, extra=None):
    out = {}

    def run():
        out["r"] = q.eig(A, fraction=f, opts=opts, return_info=True)

    med, ts = _time_calls(torch, run, warmup, steps)
    w, V, info = out["r"]
    k = len(w)
    exact = torch.as_tensor(np.sort(lam)[::-1][:k].copy(), device=A.device)
    norm = float(np.max(np.abs(lam)))
    res = float((A @ V - V * w[None, :]).norm(dim=0).max()) / norm
    orth = float((V.t() @ V - torch.eye(k, dtype=V.dtype, device=V.device)).abs().max())
    rel = float(((w - exact).abs() / exact.abs()).max())
    e = {"workload": name, "ms": med, "ms_all": [round(t, 2) for t in ts], "k": k, "ell": info["ell"],
         "kinds": info["kinds"], "rr_split": info["rr_split"], "jacobi_sweeps": info["jacobi_sweeps"],
         "mfma_frac_table1": info["flops_table1"] / (med * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
         "max_rel_value_err": rel, "residual_all_k": res, "orth_all_k": orth,
         "phases_ms": dict(zip(PHASES, [round(x, 2) for x in info["ms"]]))}
    if extra:
        e.update(extra)
    return e


def heig_entry(q, torch, name, A, lam, f, opts=None, warmup=1, steps=2):
    """Complex Hermitian solve (qdwhp_heig) timed and checked over all k vectors."""
    out = {}

    def run():
        out["r"] = q.eig_hermitian(A, f, opts=opts, return_info=True)

    med, ts = _time_calls(torch, run, warmup, steps)
    w, V, info = out["r"]
    k = len(w)
    exact = torch.as_tensor(np.sort(lam)[::-1][:k].copy(), device=A.device)
    norm = float(np.max(np.abs(lam)))
    res = float((A @ V - V * w[None, :].to(V.dtype)).norm(dim=0).max()) / norm
    orth = float((V.conj().t() @ V - torch.eye(k, dtype=V.dtype, device=V.device)).abs().max())
    rel = float(((w - exact).abs() / exact.abs()).max())
    return {"workload": name, "ms": med, "ms_all": [round(t, 2) for t in ts], "k": k,
            "ell_embedding": info["ell"], "kinds": info["kinds"], "rr_split": info["rr_split"],
            "max_rel_value_err": rel, "residual_all_k": res, "orth_all_k": orth,
            "phases_ms": dict(zip(PHASES, [round(x, 2) for x in info["ms"]])),
            "note": "solved as the 2n x 2n real symmetric embedding"}


def svd_entry(q, torch, name, A, sig, k, opts=None, warmup=1, steps=2, ref=None, extra=None):
    out = {}

    def run():
        out["r"] = q.svd(A, k, opts=opts, return_info=True)

    med, ts = _time_calls(torch, run, warmup, steps)
    U, S, V, info = out["r"]
    exact = torch.as_tensor(np.asarray(sig)[:k].copy(), device=A.device)
    r1 = (A @ V - U * S[None, :]).norm(dim=0).max()
    r2 = (A.t() @ U - V * S[None, :]).norm(dim=0).max()
    eye = torch.eye(k, dtype=U.dtype, device=U.device)
    e = {"workload": name, "ms": med, "ms_all": [round(t, 2) for t in ts], "k": k, "ell": info["ell"],
         "kinds": info["kinds"], "s": info["s"],
         "mfma_frac_table1": info["flops_table1"] / (med * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
         "max_rel_value_err": float(((S - exact).abs() / exact).max()),
         "residual_all_k": float(max(r1, r2)) / float(sig[0]),
         "orth_all_k": float(max((U.t() @ U - eye).abs().max(), (V.t() @ V - eye).abs().max())),
         "phases_ms": dict(zip(PHASES, [round(x, 2) for x in info["ms"]]))}
    if ref is not None:
        U0, S0, V0 = ref
        e["vs_fp64"] = {"max_rel_value_diff": float(((S - S0).abs() / S0).max()),
                        "max_vector_diff": float(max((U - U0).norm(dim=0).max(), (V - V0).norm(dim=0).max()))}
    if extra:
        e.update(extra)
    return e, (U, S, V)


def workloads_leg(q, torch, dev, A16, lam16):
    """The other benchmark configurations, each timed and checked."""
    from synthetic import svd_geometric, svd_loguniform, eig_uniform, CONFIG_SEEDS
    out = []
    print("[bench] eig16384 top 1%", file=sys.stderr, flush=True)
    out.append(eig_entry(q, torch, "eig16384_top1pct_clustered", A16, lam16, 0.01))
    print("[bench] eig16384 top 20% with Zolotarev steps (r = 2)", file=sys.stderr, flush=True)
    out.append(eig_entry(q, torch, "eig16384_top20pct_clustered_zolo_r2", A16, lam16, 0.2,
                         opts=q.default_opts(zolo_r=2)))
    print("[bench] svd4096 kappa 1e16 top 5%", file=sys.stderr, flush=True)
    A, sig = svd_geometric(4096, 4096, CONFIG_SEEDS["svd4096"], kappa=1e16, device=dev)
    out.append(svd_entry(q, torch, "svd4096_kappa1e16_top5pct", A, sig, 205, steps=3)[0])
    out.append(svd_entry(q, torch, "svd4096_kappa1e16_top5pct_qr_first", A, sig, 205, steps=3,
                         opts=q.default_opts(svd_qr_first=1))[0])
    out.append(svd_entry(q, torch, "svd4096_kappa1e16_top5pct_zolo_r8", A, sig, 205, steps=3,
                         opts=q.default_opts(zolo_r=8))[0])
    del A
    print("[bench] svd16384x8192 top 10%", file=sys.stderr, flush=True)
    A, sig = svd_loguniform(16384, 8192, CONFIG_SEEDS["svd16384x8192"], device=dev)
    e64, ref = svd_entry(q, torch, "svd16384x8192_top10pct_fp64", A, sig, 819, steps=3)
    out.append(e64)
    emx, _ = svd_entry(q, torch, "svd16384x8192_top10pct_mixed_fp32", A, sig, 819, steps=3,
                       opts=q.default_opts(precision=q.MIXED_FP32), ref=ref)
    emx["speedup_vs_fp64"] = e64["ms"] / emx["ms"]
    out.append(emx)
    del A, ref
    print("[bench] complex Hermitian 4096 top 10%", file=sys.stderr, flush=True)
    from synthetic import heig_clustered
    Ah, lamh = heig_clustered(4096, CONFIG_SEEDS["eig16384"], device=dev)
    out.append(heig_entry(q, torch, "heig4096_top10pct_clustered_complex", Ah, lamh, 0.1))
    del Ah
    print("[bench] eig512 top 10%", file=sys.stderr, flush=True)
    A, lam = eig_uniform(512, CONFIG_SEEDS["eig512"], device=dev)
    out.append(eig_entry(q, torch, "eig512_top10pct_uniform", A, lam, 0.1, steps=5))
    torch.cuda.synchronize()
    return out


PHASES = ["estimator", "iterations", "projector_qr", "q2", "rr_products", "small_solve", "vectors", "total"]


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
    if args.input:
        print(f"[bench] loading {args.input}", file=sys.stderr, flush=True)
        Ah = np.load(args.input, mmap_mode="r")
        lam = np.load(args.input.replace(".npy", "_lam.npy"))
        A = torch.from_numpy(np.ascontiguousarray(Ah)).to(dev)
        n = A.shape[0]
    else:
        print(f"[bench] generating n={n} planted matrix", file=sys.stderr, flush=True)
        A, lam = eig_clustered(n, 1002, device=dev)
        A = A.contiguous()              # symmetric: row-major storage is the column-major matrix
    if args.write_input:
        np.save(args.write_input, A.cpu().numpy())
        np.save(args.write_input.replace(".npy", "_lam.npy"), lam)
        print(json.dumps({"written": args.write_input, "n": n}), flush=True)
        return
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
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        solve()
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    d = info.as_dict()
    # roofline of the GEMM kernel: one more solve with per-launch events
    gflops, gms, glaunch = 0.0, 0.0, 0
    if not args.no_roofline:
        q.profile_begin()
        solve()
        torch.cuda.synchronize()
        gflops, gms, glaunch = q.profile_end()
        print("[bench] roofline pass done", file=sys.stderr, flush=True)

    # accuracy of the timed solve: planted values, every returned vector
    exact = np.sort(lam)[::-1][:k]
    wv = w.cpu().numpy()
    rel = float(np.max(np.abs(wv - exact) / np.abs(exact)))
    V = Vb.t()
    resid = float((A @ V - V * w[None, :]).norm(dim=0).max()) / float(np.max(np.abs(lam)))
    orth = float((Vb @ V - torch.eye(k, dtype=V.dtype, device=dev)).abs().max())

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
        "phases_ms": dict(zip(PHASES, [round(x, 2) for x in d["ms"]])),
        "solver": {kk: d[kk] for kk in ["ell", "ind", "kinds", "jacobi_sweeps", "rr_split", "tau", "retries"]},
        "accuracy": {"max_rel_value_err": rel, "residual_all_k": resid, "orth_all_k": orth},
        "roofline": {"bound": "mfma", "kernel": "dgemm_kernel (FP64 v_mfma_f64_16x16x4f64)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_from_profile(),
                     "traffic_unit": "HBM bytes per launch",
                     "launches": glaunch, "kernel_ms_per_solve": gms,
                     "algorithmic_flops_per_launch": gflops / max(glaunch, 1),
                     "measured": "hipEvents around each launch during one extra solve after the timed steps"},
    }
    del ws
    torch.cuda.empty_cache()
    if not args.no_workloads:
        out["workloads"] = workloads_leg(q, torch, dev, A, lam)
    del A, Vb
    torch.cuda.empty_cache()
    if not args.no_serve:
        from synthetic import request_trace, CONFIG_SEEDS
        trace = request_trace(args.serve_requests, 1.0, CONFIG_SEEDS["trace"])
        print("[bench] building request mix", file=sys.stderr, flush=True)
        mix = build_mix(torch, trace)
        print("[bench] batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(q, torch, mix[:24])
        print("[bench] same-shape batch leg", file=sys.stderr, flush=True)
        out["batched_same_shape"] = same_shape_leg(q, torch)
        for prec, key in ((q.FP64, "serving"), (q.MIXED_FP32, "serving_mixed")):
            print(f"[bench] served leg {key}", file=sys.stderr, flush=True)
            out[key] = serve_leg(q, torch, mix, trace, prec)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, f, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
