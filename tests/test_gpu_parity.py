"""End-to-end parity of the HIP path (through the C ABI) with the CPU oracle.

Each case prints its name before the GPU call."""
import numpy as np
import pytest

import oracle
from synthetic import eig_uniform, eig_clustered, svd_geometric, svd_loguniform

pytestmark = pytest.mark.gpu

# The library's default threshold on |R_ii| (0.05) differs from the paper's
# (0.01, the oracle's default): every comparison passes tol to both sides.
TOL_LIB = 0.05


def _gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_14186_amd as q
    return torch, q


def _subspace_err(V1, V2):
    return np.linalg.norm(V1 @ (V1.T @ V2) - V2, 2)


@pytest.mark.parametrize("n,f,seed,which", [(512, 0.1, 1000, "largest"), (333, 0.2, 7, "largest"),
                                            (300, 0.05, 8, "smallest"), (130, 0.3, 9, "largest")])
def test_eig_vs_oracle(n, f, seed, which):
    torch, q = _gpu()
    A, lam = eig_uniform(n, seed)
    print(f"eig n={n} f={f} which={which}", flush=True)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, which=which,
                       opts=q.default_opts(tol=TOL_LIB), return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    r = oracle.eig_partial(A, fraction=f, which=which, tol=TOL_LIB)
    k = r["k"]
    assert info["k"] == k
    # values: oracle and planted
    exact = (np.sort(lam)[::-1] if which == "largest" else np.sort(lam))[:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    # vectors: same sign convention, compare column by column (gaps are not tiny)
    assert np.max(np.abs(V - r["V"])) < 1e-9
    # estimator agreement (both sides draw the same Philox vectors)
    assert abs(info["tau"] - r["tau"] * (1 if which == "largest" else -1)) < 1e-8
    assert info["kinds"] == [s["kind"] for s in r["sched"]]
    assert abs(info["ell"] - r["ell"]) <= 2


def test_eig_storage_orders_bitwise():
    """A symmetric A passed row-major (read in place), as a transposed view
    (in place) or strided (copied) gives bitwise the same solve, and the
    count is the library's."""
    torch, q = _gpu()
    n, f = 257, 0.15
    A, lam = eig_uniform(n, 61)
    At = torch.from_numpy(A).cuda()
    big = torch.zeros((n, n + 5), dtype=torch.float64, device="cuda")
    big[:, :n] = At
    print(f"eig storage orders n={n} f={f}", flush=True)
    outs = [q.eig(X, fraction=f, opts=q.default_opts(tol=TOL_LIB)) for X in (At, At.t(), big[:, :n])]
    assert not big[:, :n].is_contiguous()
    assert outs[0][0].shape[0] == q.lib().qdwhp_eig_count(n, f) == 39
    for w, V in outs[1:]:
        assert torch.equal(w, outs[0][0]) and torch.equal(V, outs[0][1])
    exact = np.sort(lam)[::-1][:39]
    assert np.max(np.abs(outs[0][0].cpu().numpy() - exact) / np.abs(exact)) < 1e-12


def test_eig_large_lanczos_block_vs_planted():
    """32 Lanczos runs of 100 steps: the runs' tridiagonal QR works in global
    scratch (their arrays exceed 64 KiB of LDS) instead of LDS; values and
    residuals against the planted spectrum and the oracle's."""
    torch, q = _gpu()
    n, f = 600, 0.1
    A, lam = eig_uniform(n, 62)
    print(f"eig n={n} f={f} lanczos 32 x 100", flush=True)
    opts = q.default_opts(tol=TOL_LIB, lanczos_vectors=32, lanczos_steps=100)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=opts, return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    k = info["k"]
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13 and met["orth"] < 1e-12, met
    r = oracle.eig_partial(A, fraction=f, tol=TOL_LIB)
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12


@pytest.mark.parametrize("n,f,seed,which,kind,replay", [(800, 0.2, 21, "largest", "uniform", False),
                                                        (700, 0.15, 22, "smallest", "uniform", False),
                                                        (800, 0.2, 23, "largest", "clustered", False),
                                                        (800, 0.2, 24, "largest", "clustered", True)])
def test_eig_rr_split_vs_oracle(n, f, seed, which, kind, replay):
    """The exact spectral split of the Rayleigh-Ritz matrix (a converged QDWH
    polar decomposition at a Lanczos-placed shift, Jacobi on the wanted
    block only), forced at small sizes, against the oracle (which solves the
    whole Rayleigh-Ritz matrix) and the planted spectrum.  The shift comes
    from the estimator's quadrature, or (replayed threshold, no estimator
    run) from a Lanczos run on the Rayleigh-Ritz matrix itself."""
    torch, q = _gpu()
    A, lam = (eig_uniform if kind == "uniform" else eig_clustered)(n, seed)
    print(f"eig rr split n={n} f={f} which={which} {kind} replay={replay}", flush=True)
    r = oracle.eig_partial(A, fraction=f, which=which, tol=TOL_LIB)
    opts = q.default_opts(tol=TOL_LIB, **(dict(tau=r["tau"], mu=r["mu"], rho=r["rho"]) if replay else {}))
    keys = {"rr.split_min": (64, 3000), "rr.split_pct": (100, 85)}   # forced, default
    old = {key: q.tune_get(key, d) for key, (_, d) in keys.items()}
    try:
        for key, (v, _) in keys.items():
            q.tune_set(key, v)
        w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, which=which, opts=opts, return_info=True)
        torch.cuda.synchronize()
    finally:
        for key, v in old.items():
            q.tune_set(key, v)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    k = r["k"]
    print(f"  k={k} ell={info['ell']} split={info['rr_split']} sweeps={info['jacobi_sweeps']}", flush=True)
    assert k <= info["rr_split"] < info["ell"]
    exact = (np.sort(lam)[::-1] if which == "largest" else np.sort(lam))[:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    if kind == "uniform":   # isolated eigenvalues: the vectors themselves agree
        assert np.max(np.abs(V - r["V"])) < 1e-9


@pytest.mark.parametrize("n,f,seed,kind", [(800, 0.2, 25, "uniform"), (900, 0.25, 26, "clustered")])
def test_eig_rr_second_split_vs_oracle(n, f, seed, kind):
    """The wanted block of the Rayleigh-Ritz split split once more at the
    median of its spectrum (the same QDWH split, Jacobi on both halves),
    forced at small sizes, against the oracle and the planted spectrum."""
    torch, q = _gpu()
    A, lam = (eig_uniform if kind == "uniform" else eig_clustered)(n, seed)
    print(f"eig rr second split n={n} f={f} {kind}", flush=True)
    r = oracle.eig_partial(A, fraction=f, tol=TOL_LIB)
    opts = q.default_opts(tol=TOL_LIB)
    keys = {"rr.split_min": (64, 3000), "rr.split_pct": (100, 85), "rr.split2_min": (64, 0),
            "rr.split2_pct": (0, 12)}
    old = {key: q.tune_get(key, d) for key, (_, d) in keys.items()}
    try:
        for key, (v, _) in keys.items():
            q.tune_set(key, v)
        w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=opts, return_info=True)
        torch.cuda.synchronize()
    finally:
        for key, v in old.items():
            q.tune_set(key, v)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    k = r["k"]
    print(f"  k={k} ell={info['ell']} split={info['rr_split']} sweeps={info['jacobi_sweeps']}", flush=True)
    assert k <= info["rr_split"] < info["ell"]
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    if kind == "uniform":
        assert np.max(np.abs(V - r["V"])) < 1e-9


@pytest.mark.timeout(900)
def test_eig_default_tuning_at_10240_vs_oracle():
    """Default (tuned) settings, nothing forced: n = 10240, top 20% of the
    clustered spectrum runs the 128-wide GEMM tiles, the multi-panel QR
    (Cholesky-QR panels) and the Rayleigh-Ritz solve the tuned policy picks
    (the exact split when ell reaches rr.split_min), against the oracle and
    the planted spectrum."""
    torch, q = _gpu()
    n, f = 10240, 0.2
    A, lam = eig_clustered(n, 1002)
    print(f"eig default tuning n={n} f={f}", flush=True)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=q.default_opts(tol=TOL_LIB),
                       return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    print(f"  gpu done: ell={info['ell']} split={info['rr_split']}; running the oracle", flush=True)
    r = oracle.eig_partial(A, fraction=f, tol=TOL_LIB)
    k = r["k"]
    print(f"  k={k} ell gpu {info['ell']} oracle {r['ell']}", flush=True)
    assert info["k"] == k
    # the tuned policy decides the exact split of the Rayleigh-Ritz matrix
    ell = info["ell"]
    margin = max(16, k // 32)
    wants_split = ell >= q.tune_get("rr.split_min", 3000) and 100 * (k + margin) <= q.tune_get("rr.split_pct", 85) * ell
    print(f"  split wanted by the tuned policy: {wants_split}", flush=True)
    if wants_split:
        assert k <= info["rr_split"] < ell
    else:
        assert info["rr_split"] == 0
    assert abs(info["tau"] - r["tau"]) < 1e-8
    assert info["kinds"] == [st["kind"] for st in r["sched"]]
    assert abs(info["ell"] - r["ell"]) <= 2
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    # eigenvalues isolated by more than 1e-6 of the spread (the uniform part
    # of the spectrum): the vectors themselves agree
    gaps = np.minimum(np.abs(np.diff(np.concatenate([[np.inf], r["w"]]))),
                      np.abs(np.diff(np.concatenate([r["w"], [-np.inf]]))))
    sel = gaps > 2e-6
    assert sel.sum() > k // 4
    assert np.max(np.abs(V[:, sel] - r["V"][:, sel])) < 1e-7


def test_eig_replay_intermediates():
    """Same tau / mu / rho / kinds on both sides: ell and Ritz values agree."""
    torch, q = _gpu()
    A, lam = eig_clustered(600, 44)
    r = oracle.eig_partial(A, fraction=0.1, tol=TOL_LIB)
    o = q.default_opts(tol=TOL_LIB, tau=r["tau"], mu=r["mu"], rho=r["rho"], kinds=[s["kind"] for s in r["sched"]])
    print("eig replay n=600", flush=True)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=0.1, opts=o, return_info=True)
    assert info["ell"] == r["ell"] and info["ind"] == r["ind"]
    assert np.max(np.abs(w.cpu().numpy() - r["w"]) / np.abs(r["w"])) < 1e-12
    # clustered top eigenvalues: compare the spanned subspace
    assert _subspace_err(V.cpu().numpy(), r["V"]) < 1e-10


@pytest.mark.parametrize("m,n,k,kind", [(512, 512, 26, "geo"), (400, 250, 25, "log"),
                                        (250, 400, 25, "log"), (300, 300, 15, "geo")])
def test_svd_vs_oracle(m, n, k, kind):
    torch, q = _gpu()
    if kind == "geo":
        A, sig = svd_geometric(m, n, 1001)
    else:
        A, sig = svd_loguniform(max(m, n), min(m, n), 1003)
        if m < n:
            A = A.T.copy()
    print(f"svd m={m} n={n} k={k}", flush=True)
    U, S, V, info = q.svd(torch.from_numpy(A).cuda(), k, opts=q.default_opts(tol=TOL_LIB), return_info=True)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    r = oracle.svd_partial(A, k, tol=TOL_LIB)
    assert np.max(np.abs(S - r["S"]) / r["S"]) < 1e-12
    assert np.max(np.abs(S - sig[:k]) / sig[:k]) < 1e-12
    met = oracle.svd_metrics(A, U, S, V, sig[:k])
    assert met["residual"] < 1e-13, met
    assert max(met["orth_u"], met["orth_v"]) < 1e-12, met
    assert np.max(np.abs(V - r["V"])) < 1e-8 and np.max(np.abs(U - r["U"])) < 1e-8
    assert info["kinds"] == [s["kind"] for s in r["sched"]]


@pytest.mark.parametrize("m,n,k", [(900, 600, 30), (640, 640, 32)])
def test_structured_stacked_qr_vs_full_and_oracle(m, n, k):
    """The QR of [sqrt(c) X; I] that skips the identity rows no reflector
    has reached yet (the structure of the stacked matrix) against the QR of
    the full stacked matrix and the oracle, on an SVD whose first step is
    QR-based (svd_qr_first = 1) and kappa = 1e16."""
    torch, q = _gpu()
    A, sig = svd_geometric(m, n, 1005, kappa=1e16)
    print(f"structured stacked qr m={m} n={n} k={k}", flush=True)
    o = q.default_opts(tol=TOL_LIB, svd_qr_first=1)
    res = {}
    old = q.tune_get("qr.stacked", 1)
    try:
        for stacked in (1, 0):
            q.tune_set("qr.stacked", stacked)
            U, S, V, info = q.svd(torch.from_numpy(A).cuda(), k, opts=o, return_info=True)
            torch.cuda.synchronize()
            res[stacked] = (U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info)
    finally:
        q.tune_set("qr.stacked", old)
    r = oracle.svd_partial(A, k, tol=TOL_LIB, qr_first=True)
    assert res[1][3]["kinds"][0] == "qr" and res[1][3]["kinds"] == [st["kind"] for st in r["sched"]]
    assert res[1][3]["ell"] == res[0][3]["ell"]
    S1, S0 = res[1][1], res[0][1]
    assert np.max(np.abs(S1 - S0) / S0) < 1e-13
    assert np.max(np.abs(S1 - r["S"]) / r["S"]) < 1e-12
    assert np.max(np.abs(S1 - sig[:k]) / sig[:k]) < 1e-12
    met = oracle.svd_metrics(A, res[1][0], S1, res[1][2], sig[:k])
    assert met["residual"] < 1e-13, met
    assert max(met["orth_u"], met["orth_v"]) < 1e-12, met
    assert np.max(np.abs(res[1][2] - res[0][2])) < 1e-9


# ------------------------------------------------------- Zolotarev steps (r > 1)
@pytest.mark.parametrize("n,f,seed,r,spec", [(512, 0.1, 1000, 2, "uniform"), (600, 0.2, 41, 13, "clustered"),
                                             (700, 0.15, 42, 3, "uniform"), (400, 0.1, 43, 1, "uniform")])
def test_zolotarev_eig_vs_oracle(n, f, seed, r, spec):
    """Zolotarev steps of type (2r+1, 2r) in Algorithm 1 (r = 13 from s = 0.2:
    one step, its terms with small c_{2j-1} QR-based; r = 1: the DWH steps),
    against the oracle's Zolotarev iteration and the planted spectrum."""
    torch, q = _gpu()
    A, lam = (eig_uniform if spec == "uniform" else eig_clustered)(n, seed)
    print(f"zolotarev eig n={n} f={f} r={r} {spec}", flush=True)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=q.default_opts(tol=TOL_LIB, zolo_r=r),
                       return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    o = oracle.eig_partial(A, fraction=f, tol=TOL_LIB, zolo_r=r)
    k = o["k"]
    print(f"  steps {info['n_iter']} kinds {info['kinds']} ell {info['ell']} / {o['ell']}", flush=True)
    assert abs(info["tau"] - o["tau"]) < 1e-8
    assert info["kinds"] == [st["kind"] for st in o["sched"]]
    assert [round(x[1]) for x in info["weights"][:info["n_iter"]]] == [r] * info["n_iter"]
    assert abs(info["ell"] - o["ell"]) <= 2
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - o["w"]) / np.abs(o["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    if r == 1:     # the DWH steps with the plain threshold cut
        w0, V0, i0 = q.eig(torch.from_numpy(A).cuda(), fraction=f, return_info=True,
                           opts=q.default_opts(tol=TOL_LIB, tau_policy=0))
        assert i0["ell"] == info["ell"] and i0["kinds"] == info["kinds"]
        assert np.max(np.abs(w0.cpu().numpy() - w) / np.abs(w)) < 1e-13


@pytest.mark.parametrize("m,n,k,r,kind", [(500, 300, 15, 8, "geo"), (400, 400, 20, 3, "log"),
                                          (300, 500, 25, 2, "log")])
def test_zolotarev_svd_vs_oracle(m, n, k, r, kind):
    """Zolotarev steps in Algorithm 2: kappa = 1e16 with r = 8 (the first
    step's terms QR-based, s < 1e-3), and log-uniform spectra (wide too)."""
    torch, q = _gpu()
    if kind == "geo":
        A, sig = svd_geometric(m, n, 1011, kappa=1e16)
    else:
        A, sig = svd_loguniform(max(m, n), min(m, n), 1012)
        if m < n:
            A = A.T.copy()
    print(f"zolotarev svd m={m} n={n} k={k} r={r}", flush=True)
    U, S, V, info = q.svd(torch.from_numpy(A).cuda(), k, opts=q.default_opts(tol=TOL_LIB, zolo_r=r),
                          return_info=True)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    o = oracle.svd_partial(A, k, tol=TOL_LIB, zolo_r=r)
    print(f"  steps {info['n_iter']} kinds {info['kinds']} ell {info['ell']} / {o['ell']}", flush=True)
    assert info["kinds"] == [st["kind"] for st in o["sched"]]
    assert abs(info["ell"] - o["ell"]) <= 2
    assert np.max(np.abs(S - o["S"]) / o["S"]) < 1e-12
    assert np.max(np.abs(S - sig[:k]) / sig[:k]) < 1e-12
    met = oracle.svd_metrics(A, U, S, V, sig[:k])
    assert met["residual"] < 1e-13, met
    assert max(met["orth_u"], met["orth_v"]) < 1e-12, met


# ------------------------------------------------------------------ tol = 0.01
# The paper's threshold (Sec. 4.1, Algorithms 1 and 2) on both sides.  The
# guarantee the paper gives for the subspace is Theorem 1: sin angle(V0, Q2)
# <= ||V0^T B|| / sigma_min(R11), V0 the planted wanted vectors.  With the
# plain (non-pivoted) QR sigma_min(R11) falls well below tol (3e-4 .. 1e-3
# on the kappa = 1e16 SVD inputs), and the residuals of both sides, about
# sin angle x ||A||, land between 1e-14 and ~2e-13 depending on rounding (the
# same oracle gives 7e-14 on one host's BLAS and 1.7e-13 on another's for
# the same input).  Gate: the GPU's residual within 1e-13, or within the
# Theorem 1 bound of the oracle's own factorisation.
PAPER_CASES = [("eig", 512, 512, 0.1, 1000, "uniform"), ("eig", 1024, 1024, 0.01, 1002, "clustered"),
               ("eig", 2048, 2048, 0.2, 1002, "clustered"),
               ("svd", 300, 300, 15, 1001, "geo"), ("svd", 300, 300, 15, 1002, "geo"),
               ("svd", 300, 300, 15, 1003, "geo"), ("svd", 512, 512, 26, 1001, "geo"),
               ("svd", 512, 512, 26, 1003, "geo"), ("svd", 1024, 512, 51, 1003, "log")]


def _theorem1_bound(B, ind, V0):
    _, R = np.linalg.qr(B)
    smin = np.linalg.svd(R[:ind - 1, :ind - 1], compute_uv=False).min() if ind > 1 else 1.0
    return float(np.linalg.norm(V0.T @ B, 2) / smin)


@pytest.mark.parametrize("kind,m,n,f,seed,spec", PAPER_CASES)
def test_paper_tol_vs_oracle(kind, m, n, f, seed, spec):
    from synthetic import rng, haar
    torch, q = _gpu()
    tol = 0.01
    print(f"paper tol {kind} {m}x{n} f={f} seed={seed} {spec}", flush=True)
    o = q.default_opts(tol=tol)
    g = rng(seed)
    if kind == "eig":
        A, lam = (eig_uniform if spec == "uniform" else eig_clustered)(n, seed)
        Qp = haar(g, n)                       # the planted eigenvectors (same draws)
        w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=o, return_info=True)
        w, V = w.cpu().numpy(), V.cpu().numpy()
        r = oracle.eig_partial(A, fraction=f, tol=tol)
        k = r["k"]
        exact = np.sort(lam)[::-1][:k]
        met = oracle.eig_metrics(A, w, V, exact)
        ref = oracle.eig_metrics(A, r["w"], r["V"], exact)
        vals, rvals = w, r["w"]
        V0 = Qp[:, lam >= r["tau"]]            # the approximate null space of B
    else:
        A, sig = (svd_geometric(m, n, seed, kappa=1e16) if spec == "geo" else svd_loguniform(m, n, seed))
        haar(g, m, n)
        Vp = haar(g, n)
        U, S, V, info = q.svd(torch.from_numpy(A).cuda(), f, opts=o, return_info=True)
        U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        r = oracle.svd_partial(A, f, tol=tol)
        exact = sig[:f]
        met = oracle.svd_metrics(A, U, S, V, exact)
        ref = oracle.svd_metrics(A, r["U"], r["S"], r["V"], exact)
        vals, rvals = S, r["S"]
        V0 = Vp[:, :f]
    bound = _theorem1_bound(r["B"], r["ind"], V0)
    print(f"  ell gpu {info['ell']} oracle {r['ell']}; residual gpu {met['residual']:.2e} "
          f"oracle {ref['residual']:.2e}; Theorem 1 bound {bound:.2e}; values {met['value_rel_max']:.2e}",
          flush=True)
    assert info["kinds"] == [st["kind"] for st in r["sched"]]
    assert abs(info["ell"] - r["ell"]) <= 2
    assert np.max(np.abs(vals - rvals) / np.abs(rvals)) < 1e-12
    assert met["value_rel_max"] < 1e-12
    assert ref["residual"] <= max(1e-13, bound)
    assert met["residual"] <= max(1e-13, bound), (met, ref, bound)


# ------------------------------------------- threshold policy, Omega, s = 0.875
@pytest.mark.parametrize("n,f,seed,policy,omega", [(1024, 0.01, 1002, "cost", 0), (1024, 0.01, 1002, "plain", 0),
                                                   (512, 0.1, 1000, "plain", 0), (600, 0.1, 31, "cost", 1),
                                                   (1024, 0.01, 1002, "cost", 1)])
def test_threshold_policy_and_omega_vs_oracle(n, f, seed, policy, omega):
    """The cost-model threshold (a cut below the plain one when it turns
    QR-based steps into Cholesky-based ones) and the QR of B Omega (Sec. 4.1)
    give the oracle's threshold, kinds and subspace size, and the planted values."""
    torch, q = _gpu()
    A, lam = (eig_clustered if seed == 1002 else eig_uniform)(n, seed)
    print(f"policy {policy} omega {omega} n={n} f={f}", flush=True)
    o = q.default_opts(tol=TOL_LIB, tau_policy=1 if policy == "cost" else 0, use_omega=omega)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=o, return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    r = oracle.eig_partial(A, fraction=f, tol=TOL_LIB, tau_policy=policy, use_omega=bool(omega))
    k = r["k"]
    print(f"  tau {info['tau']:.6f} / {r['tau']:.6f} kinds {info['kinds']} ell {info['ell']} / {r['ell']}", flush=True)
    assert abs(info["tau"] - r["tau"]) < 1e-8
    assert info["kinds"] == [st["kind"] for st in r["sched"]]
    assert abs(info["ell"] - r["ell"]) <= 2
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13, met


def _tail_spectrum(n, seed):
    """10% of the eigenvalues in [0.5, 1], the rest far below in [-30, -5]:
    the unwanted side lies beyond the two-step band, where s = 0.875 pays."""
    from synthetic import rng, haar, planted_sym
    g = rng(seed)
    Q = haar(g, n)
    nt = n // 10
    lam = np.concatenate([g.uniform(0.5, 1.0, nt), g.uniform(-30.0, -5.0, n - nt)])
    return planted_sym(Q, lam), lam


@pytest.mark.parametrize("n,f,seed,spec", [(512, 0.1, 1000, "uniform"), (600, 0.08, 33, "tail")])
def test_two_step_variant_vs_oracle(n, f, seed, spec):
    """Sec. 4.1's other shift choice: s = 0.875 with two DWH steps (type (9,8)):
    cheaper iterations, a band reaching ~5 |mu| beyond the threshold (on a
    uniform spectrum that is everything, ell = n; with the unwanted part far
    below, ell stays near k)."""
    torch, q = _gpu()
    A, lam = eig_uniform(n, seed) if spec == "uniform" else _tail_spectrum(n, seed)
    print(f"s=0.875 two steps n={n} f={f} {spec}", flush=True)
    o = q.default_opts(tol=TOL_LIB, s_eig=0.875, eig_iters=2)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=f, opts=o, return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    r = oracle.eig_partial(A, fraction=f, tol=TOL_LIB, s=0.875, iters=2)
    k = r["k"]
    print(f"  kinds {info['kinds']} ell {info['ell']} / {r['ell']}", flush=True)
    assert info["n_iter"] == 2 and info["kinds"] == [st["kind"] for st in r["sched"]]
    assert abs(info["ell"] - r["ell"]) <= 2
    if spec == "tail":
        assert info["ell"] < n // 2
    exact = np.sort(lam)[::-1][:k]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    met = oracle.eig_metrics(A, w, V, exact)
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13, met


# ------------------------------------------- QDWH-SVD small solve (f1, SVD side)
@pytest.mark.parametrize("m,n,k,kind", [(600, 400, 40, "log"), (512, 512, 26, "geo"), (400, 700, 35, "log")])
def test_svd_polar_small_solve_vs_oracle(m, n, k, kind):
    """The SVD of the Rayleigh-Ritz factor R_Y by QDWH-SVD (Sec. 3.2: a
    converged QDWH polar decomposition R_Y = U_p H, then the symmetric
    eigenproblem of H), forced at small sizes, against the oracle (LAPACK SVD
    of R_Y) and the planted singular values."""
    torch, q = _gpu()
    if kind == "geo":
        A, sig = svd_geometric(m, n, 1001)
    else:
        A, sig = svd_loguniform(max(m, n), min(m, n), 1003)
        if m < n:
            A = A.T.copy()
    print(f"svd polar small solve m={m} n={n} k={k}", flush=True)
    old = q.tune_get("rr.svd_polar", 256)
    try:
        q.tune_set("rr.svd_polar", 32)
        U, S, V, info = q.svd(torch.from_numpy(A).cuda(), k, opts=q.default_opts(tol=TOL_LIB), return_info=True)
        torch.cuda.synchronize()
    finally:
        q.tune_set("rr.svd_polar", old)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    r = oracle.svd_partial(A, k, tol=TOL_LIB)
    print(f"  ell={info['ell']} sweeps={info['jacobi_sweeps']}", flush=True)
    assert np.max(np.abs(S - r["S"]) / r["S"]) < 1e-12
    met = oracle.svd_metrics(A, U, S, V, sig[:k])
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13, met
    assert max(met["orth_u"], met["orth_v"]) < 1e-12, met
    assert np.max(np.abs(V - r["V"])) < 1e-8 and np.max(np.abs(U - r["U"])) < 1e-8
