"""Autotuner for the launch-shape parameters of libqdwhp.so on this GPU.

    python -m paper_2104_14186_amd.autotune [--out PATH]

Measures, on the device, the candidates of each tuning key and writes the
winners (plus the measurements behind them) as JSON; the binding loads
the file at library load (tuning_gfx950.json beside this module) and hands
each key to qdwhp_tune_set.  None of the keys changes results, only speed:
  gemm.small_tiles  -- a GEMM launch with fewer 128x128 tiles than this runs
                       64x64 tiles; swept over square products n^3 and the
                       tall-skinny shapes of the estimator and projections;
  batch.lanes       -- concurrent streams of qdwhp_batched, swept on a ragged
                       batch drawn like the served request mix;
  serve.lanes       -- the same choice for the request server.
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


def tune_lanes(q, torch, log, count=24, seed=7):
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
    rows = []
    for lanes in (1, 2, 4, 8, 12, 16):
        t = _time(lambda: q.batched(specs, lanes=lanes), 1, torch)
        rows.append(dict(lanes=lanes, s=t, solves_per_s=count / t))
        log(f"batch lanes={lanes}: {t*1e3:.1f} ms for {count} problems ({count / t:.1f} solves/s)")
    best = min(rows, key=lambda r: r["s"])["lanes"]
    return best, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    import paper_2104_14186_amd as q
    q.lib()
    q.lib().qdwhp_tune_clear()
    log = lambda s: print("[autotune] " + s, flush=True)
    small, grows = tune_gemm(q, torch, log)
    q.tune_set("gemm.small_tiles", small)
    lanes, lrows = tune_lanes(q, torch, log)
    out = {"device": torch.cuda.get_device_name(0),
           "params": {"gemm.small_tiles": small, "batch.lanes": lanes, "serve.lanes": lanes},
           "gemm": grows, "lanes": lrows}
    path = args.out or q.TUNING_PATH
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {path}: {out['params']}")


if __name__ == "__main__":
    main()
