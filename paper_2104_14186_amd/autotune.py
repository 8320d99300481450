"""Autotuner for the launch-shape parameters of libqdwhp.so on this GPU.

    python -m paper_2104_14186_amd.autotune [--out PATH] [--quick]

Measures, on the device, the candidates of each tuning key and writes the
winners (plus the measurements behind them) as JSON; the binding loads
the file at library load (tuning_gfx950.json beside this module) and hands
each key to qdwhp_tune_set.  None of the keys changes the method's results
beyond rounding order (most not even that), only speed.  Keys by kernel,
size bucket and precision:
  gemm.small_tiles   -- FP64 GEMM: a launch with fewer 128x128 tiles than this
                        runs 64x64 tiles; swept over square products and the
                        tall-skinny shapes of the estimator and projections;
  gemm.shallow_k     -- FP64 GEMM: launches with k at most this run 64x64
                        tiles (block-reflector updates); swept over k;
  qr.recon@b         -- Householder QR, per panel-height bucket b =
                        ceil(log2 h): Cholesky-QR panels with Householder
                        reconstruction (1) or one launch per column (0);
  jacobi.fused_max   -- two-sided Jacobi: sizes up to this update H and V in
                        one launch per round (above: helper stream);
  dc.leaf            -- full-spectrum divide and conquer: leaf size;
  rr.svd_polar       -- SVD Rayleigh-Ritz factors from this many rows up go
                        the QDWH-SVD way (polar decomposition + eig);
  rr.split_min       -- EIG Rayleigh-Ritz matrices from this many rows up are
                        split exactly before Jacobi;
  batch.lanes,       -- concurrent streams of qdwhp_batched (FP64 and mixed
  batch.lanes.mixed     precision), swept on a ragged batch drawn like the
                        served request mix;
  serve.lanes        -- the request server's lanes: the FP64 batch choice,
                        capped at 3 so that with the caller's stream the
                        process stays within its 4 hardware queues.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune_gemm(q, torch, log):
    """Per shape, time 128- and 64-wide tiles; the threshold is the smallest
    128-tile count at which 128 wins for every larger shape."""
    shapes = []
    for n in (128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072):
        shapes.append((n, n, n))
    for n in (512, 1024, 2048, 4096, 8192):
        shapes.append((n, 8, n))          # estimator operator (n x nv)
        shapes.append((n, n // 8, n))     # projections onto a subspace
    rows = []
    for (m, nn, k) in shapes:
        A = torch.randn(k, m, dtype=torch.float64, device="cuda")
        B = torch.randn(nn, k, dtype=torch.float64, device="cuda")
        C = torch.zeros(nn, m, dtype=torch.float64, device="cuda")
        t = {}
        for name, thr in (("t128", 0), ("t64", 1 << 40)):
            q.tune_set("gemm.small_tiles", thr)
            reps = max(3, min(200, int(2e10 / (2.0 * m * nn * k + 1))))
            t[name] = _time(lambda: q.dgemm(A, B, C), reps, torch)
        tiles = math.ceil(m / 128) * math.ceil(nn / 128)
        rows.append(dict(m=m, n=nn, k=k, tiles128=tiles, ms128=t["t128"] * 1e3, ms64=t["t64"] * 1e3))
        log(f"gemm {m}x{nn}x{k} tiles128={tiles} 128:{t['t128']*1e3:.3f} ms 64:{t['t64']*1e3:.3f} ms")
    # smallest threshold T such that shapes with tiles128 < T prefer 64 (count wins)
    cands = sorted({r["tiles128"] for r in rows} | {1 << 30})
    best, best_cost = 1, None
    for T in [1] + [c + 1 for c in cands]:
        cost = sum(r["ms64"] if r["tiles128"] < T else r["ms128"] for r in rows)
        if best_cost is None or cost < best_cost - 1e-9:
            best, best_cost = T, cost
    return best, rows


def tune_shallow_k(q, torch, log, quick=False):
    """Per depth k, 128- against 64-wide tiles for a wide update
    C (m x n) += A (m x k) B (k x n); the threshold is the largest k at
    which 64 still wins (0: never)."""
    m = n = 4096 if quick else 8192
    rows = []
    for k in (32, 64, 128, 256, 512):
        A = torch.randn(k, m, dtype=torch.float64, device="cuda")
        B = torch.randn(n, k, dtype=torch.float64, device="cuda")
        C = torch.zeros(n, m, dtype=torch.float64, device="cuda")
        t = {}
        q.tune_set("gemm.small_tiles", 0)
        for name, sk in (("t128", 0), ("t64", 1 << 30)):
            q.tune_set("gemm.shallow_k", sk)
            t[name] = _time(lambda: q.dgemm(A, B, C), 10, torch)
        rows.append(dict(m=m, n=n, k=k, ms128=t["t128"] * 1e3, ms64=t["t64"] * 1e3))
        log(f"shallow gemm {m}x{n}x{k}: 128:{t['t128']*1e3:.3f} ms 64:{t['t64']*1e3:.3f} ms")
    best = 0
    for r in rows:
        if r["ms64"] < r["ms128"]:
            best = r["k"]
        else:
            break
    return best, rows


def tune_qr_recon(q, torch, log, quick=False):
    """Per size bucket, Cholesky-QR panels against per-column launches."""
    rows, params = [], {}
    for n in ((256, 1024, 4096) if quick else (128, 256, 512, 1024, 2048, 4096, 8192)):
        A = torch.randn(n, n, dtype=torch.float64, device="cuda")
        t = {}
        for rc in (1, 0):
            q.tune_set("qr.recon", rc)
            t[rc] = _time(lambda: q.qr(A), 3 if n >= 4096 else 10, torch)
        b = max(0, math.ceil(math.log2(n)))
        params[f"qr.recon@{b}"] = 1 if t[1] <= t[0] else 0
        rows.append(dict(n=n, bucket=b, ms_recon=t[1] * 1e3, ms_columns=t[0] * 1e3))
        log(f"qr {n}x{n}: recon {t[1]*1e3:.2f} ms, column steps {t[0]*1e3:.2f} ms")
    q.tune_set("qr.recon", 1)
    return params, rows


def tune_fused(q, torch, log, quick=False):
    """Two-sided Jacobi: one launch per round against the helper stream."""
    rows = []
    for n in ((512, 2048) if quick else (256, 512, 768, 1024, 1536, 2048, 3072)):
        G = torch.randn(n, n, dtype=torch.float64, device="cuda")
        H = 0.5 * (G + G.t())
        t = {}
        for name, fm in (("fused", n), ("stream", n - 1)):
            q.tune_set("jacobi.fused_max", fm)
            t[name] = _time(lambda: q.syev(H), 1, torch)
        rows.append(dict(n=n, ms_fused=t["fused"] * 1e3, ms_stream=t["stream"] * 1e3))
        log(f"syev {n}: fused {t['fused']*1e3:.1f} ms, helper stream {t['stream']*1e3:.1f} ms")
    best = 0                     # the largest n up to which the one-launch rounds win at every size
    for r in rows:
        if r["ms_fused"] <= r["ms_stream"]:
            best = r["n"]
        else:
            break
    return best, rows


def tune_dc_leaf(q, torch, log, quick=False):
    n = 1024 if quick else 2048
    G = torch.randn(n, n, dtype=torch.float64, device="cuda")
    H = 0.5 * (G + G.t())
    rows = []
    for leaf in (128, 256, 512, 1024):
        q.tune_set("dc.leaf", leaf)
        t = _time(lambda: q.syev_dc(H), 1, torch)
        rows.append(dict(n=n, leaf=leaf, ms=t * 1e3))
        log(f"syev_dc {n} leaf {leaf}: {t*1e3:.1f} ms")
    return min(rows, key=lambda r: r["ms"])["leaf"], rows


def _phase(info, name):
    names = ["estimator", "iterations", "projector_qr", "q2", "rr_products", "small_solve", "vectors", "total"]
    return info["ms"][names.index(name)]


def tune_svd_polar(q, torch, log, quick=False):
    """Small SVD solve by one-sided Jacobi against the polar route, by the
    Rayleigh-Ritz factor's size ell; the threshold is the smallest ell from
    which the polar route wins at every measured larger size."""
    from synthetic import svd_loguniform
    rows = []
    for n, f in (((1024, 0.1), (2048, 0.1)) if quick else ((1024, 0.1), (2048, 0.1), (4096, 0.1), (8192, 0.1))):
        A, _ = svd_loguniform(n, n, 3100 + n, device=torch.device("cuda"))
        k = max(1, int(f * n + 0.5))
        t, ell = {}, 0
        for name, thr in (("polar", 1), ("jacobi", 1 << 30)):
            q.tune_set("rr.svd_polar", thr)
            q.svd(A, k, return_info=True)
            torch.cuda.synchronize()
            _, _, _, info = q.svd(A, k, return_info=True)
            t[name] = _phase(info, "small_solve")
            ell = info["ell"]
        rows.append(dict(n=n, ell=ell, ms_polar=t["polar"], ms_jacobi=t["jacobi"]))
        log(f"svd {n} (ell {ell}): small solve polar {t['polar']:.1f} ms, Jacobi {t['jacobi']:.1f} ms")
    rows.sort(key=lambda r: r["ell"])
    best = 1 << 30
    for r in reversed(rows):
        if r["ms_polar"] < r["ms_jacobi"]:
            best = r["ell"]
        else:
            break
    return best, rows


def tune_split(q, torch, log, quick=False):
    """Exact split of the EIG Rayleigh-Ritz matrix against Jacobi on all of
    it, by ell; the threshold is the smallest ell from which the split wins."""
    from synthetic import eig_clustered
    rows = []
    for n in ((8192,) if quick else (6144, 8192, 10240, 12288)):
        A, _ = eig_clustered(n, 3200 + n, device=torch.device("cuda"))
        t, ell = {}, 0
        for name, thr in (("split", 64), ("jacobi", 1 << 30)):
            q.tune_set("rr.split_min", thr)
            q.eig(A, fraction=0.2, return_info=True)
            torch.cuda.synchronize()
            _, _, info = q.eig(A, fraction=0.2, return_info=True)
            t[name] = _phase(info, "small_solve")
            ell = info["ell"]
        rows.append(dict(n=n, ell=ell, ms_split=t["split"], ms_jacobi=t["jacobi"]))
        log(f"eig {n} 20% (ell {ell}): small solve split {t['split']:.1f} ms, Jacobi {t['jacobi']:.1f} ms")
        del A
    rows.sort(key=lambda r: r["ell"])
    best = 1 << 30
    for r in reversed(rows):
        if r["ms_split"] < r["ms_jacobi"]:
            best = r["ell"]
        else:
            break
    return best, rows


def tune_split2(q, torch, log, quick=False):
    """One more split of the wanted block (when it is clustered) against
    Jacobi on all of it, by the wanted block's rows r; the threshold is the
    smallest r from which the second split wins."""
    from synthetic import eig_clustered
    rows = []
    for n in ((12288,) if quick else (10240, 12288, 16384)):
        A, _ = eig_clustered(n, 3300 + n, device=torch.device("cuda"))
        t, r = {}, 0
        for name, thr in (("split2", 64), ("jacobi", 0)):
            q.tune_set("rr.split2_min", thr)
            q.eig(A, fraction=0.2, return_info=True)
            torch.cuda.synchronize()
            _, _, info = q.eig(A, fraction=0.2, return_info=True)
            t[name] = _phase(info, "small_solve")
            r = info["rr_split"]
        rows.append(dict(n=n, r=r, ms_split2=t["split2"], ms_jacobi=t["jacobi"]))
        log(f"eig {n} 20% (wanted block {r}): small solve second split {t['split2']:.1f} ms, "
            f"Jacobi {t['jacobi']:.1f} ms")
        del A
        torch.cuda.empty_cache()
    rows.sort(key=lambda x: x["r"])
    best = 0
    for x in reversed(rows):
        if x["r"] > 0 and x["ms_split2"] < x["ms_jacobi"]:
            best = x["r"]
        else:
            break
    return best, rows


def tune_lanes(q, torch, log, count=24, seed=7, precision=None):
    from synthetic import eig_uniform, svd_geometric
    import numpy as np
    g = np.random.default_rng(seed)
    dev = torch.device("cuda")
    specs = []
    for i in range(count):
        n = int(g.choice([256, 512, 1024, 2048]))
        f = float(g.uniform(0.01, 0.2))
        if g.uniform() < 0.6:
            specs.append(dict(type="eig", A=eig_uniform(n, 9000 + i, device=dev)[0], fraction=f))
        else:
            A = svd_geometric(n, n, 9000 + i, kappa=10 ** g.uniform(0, 12), device=dev)[0]
            specs.append(dict(type="svd", A=A, k=max(1, int(f * n + 0.5))))
    opts = q.default_opts(precision=precision) if precision is not None else None
    rows = []
    for lanes in (1, 2, 4, 8):
        t = _time(lambda: q.batched(specs, lanes=lanes, opts=opts), 1, torch)
        rows.append(dict(lanes=lanes, s=t, solves_per_s=count / t))
        log(f"batch lanes={lanes}{' (mixed)' if precision is not None else ''}: "
            f"{t*1e3:.1f} ms for {count} problems ({count / t:.1f} solves/s)")
    best = min(rows, key=lambda r: r["s"])["lanes"]
    return best, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true", help="fewer sizes per sweep")
    ap.add_argument("--only", choices=["split2"], default=None,
                    help="run one sweep on top of the committed table and update it")
    args = ap.parse_args()
    import torch
    import paper_2104_14186_amd as q
    q.lib()
    log = lambda s: print("[autotune] " + s, flush=True)
    if args.only == "split2":
        path = args.out or q.TUNING_PATH
        table = json.load(open(q.TUNING_PATH))
        s2, table["rr_split2"] = tune_split2(q, torch, log, args.quick)
        table["params"]["rr.split2_min"] = s2
        with open(path, "w") as f:
            json.dump(table, f, indent=1)
        log(f"wrote {path}: rr.split2_min = {s2}")
        return
    q.lib().qdwhp_tune_clear()
    params, meas = {}, {}
    small, meas["gemm"] = tune_gemm(q, torch, log)
    params["gemm.small_tiles"] = small
    q.tune_set("gemm.small_tiles", small)
    sk, meas["gemm_shallow"] = tune_shallow_k(q, torch, log, args.quick)
    params["gemm.shallow_k"] = sk
    q.tune_set("gemm.small_tiles", small)
    q.tune_set("gemm.shallow_k", sk)
    qr_params, meas["qr"] = tune_qr_recon(q, torch, log, args.quick)
    params.update(qr_params)
    for key, v in qr_params.items():
        q.tune_set(key, v)
    fm, meas["jacobi_fused"] = tune_fused(q, torch, log, args.quick)
    params["jacobi.fused_max"] = fm
    q.tune_set("jacobi.fused_max", fm)
    leaf, meas["dc_leaf"] = tune_dc_leaf(q, torch, log, args.quick)
    params["dc.leaf"] = leaf
    q.tune_set("dc.leaf", leaf)
    pol, meas["svd_polar"] = tune_svd_polar(q, torch, log, args.quick)
    params["rr.svd_polar"] = pol
    q.tune_set("rr.svd_polar", pol)
    spl, meas["rr_split"] = tune_split(q, torch, log, args.quick)
    params["rr.split_min"] = spl
    q.tune_set("rr.split_min", spl)
    s2, meas["rr_split2"] = tune_split2(q, torch, log, args.quick)
    params["rr.split2_min"] = s2
    q.tune_set("rr.split2_min", s2)
    lanes, meas["lanes"] = tune_lanes(q, torch, log)
    lanes_mx, meas["lanes_mixed"] = tune_lanes(q, torch, log, precision=q.MIXED_FP32)
    params.update({"batch.lanes": lanes, "batch.lanes.mixed": lanes_mx, "serve.lanes": min(lanes, 3)})
    out = {"device": torch.cuda.get_device_name(0), "params": params, **meas}
    path = args.out or q.TUNING_PATH
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {path}: {out['params']}")


if __name__ == "__main__":
    main()
