"""Pins of the oracle's matrix-level steps and of Algorithms 1 and 2 against
closed forms, invariants, planted spectra and brute-force Jacobi."""
import math

import numpy as np
import pytest

import oracle
from oracle.dwh import dwh_weights, compose, svd_schedule
from oracle.polar import qr_step, chol_step, halley_direct_step
from oracle.partial import projector_subspace, NoSubspace
from oracle.estimator import lanczos_slq, count_above
from synthetic import rng, haar, planted_sym, planted_general, eig_uniform, eig_clustered, \
    svd_geometric, svd_loguniform


def _rand_X(m, n, lo, seed):
    g = rng(seed)
    U, V = haar(g, m, n), haar(g, n)
    sig = np.geomspace(lo, 1.0, n)
    return planted_general(U, sig, V), U, sig, V


@pytest.mark.parametrize("l,m,n", [(0.2, 40, 30), (0.05, 64, 64), (1e-3, 50, 20)])
def test_three_forms_of_one_step_agree(l, m, n):
    """Eq. (1), Eq. (2) and Eq. (3) are the same map in exact arithmetic; each
    is compared with the planted closed form U r(Sigma) V^T.  Eq. (2) is
    backward stable; the other two lose accuracy with cond(I + c X^T X) <= 1 + c."""
    X, U, sig, V = _rand_X(m, n, l, 7)
    a, b, c = dwh_weights(l)
    closed = planted_general(U, compose(sig, [(a, b, c)]), V)
    nx = np.linalg.norm(closed)
    assert np.linalg.norm(qr_step(X, a, b, c) - closed) / nx < 1e-14
    for fn in (chol_step, halley_direct_step):
        assert np.linalg.norm(fn(X, a, b, c) - closed) / nx < 1e-15 * (1 + c) * 4


def test_higham_identity():
    """Sec. 3.1: c X (I + c^2 X^T X)^{-1} = Q1 Q2^T for [cX; I] = [Q1; Q2] R."""
    g = rng(3)
    X = g.standard_normal((30, 12))
    for c in [0.3, 2.0, 11.0]:
        Q, _ = np.linalg.qr(np.vstack([c * X, np.eye(12)]))
        lhs = c * X @ np.linalg.inv(np.eye(12) + c * c * X.T @ X)
        assert np.linalg.norm(lhs - Q[:30] @ Q[30:].T) / np.linalg.norm(lhs) < 1e-14


@pytest.mark.parametrize("step", ["qr", "chol"])
def test_iterates_match_scalar_composite(step):
    """Sec. 3.1: after k steps X_k = U r_k(...r_1(Sigma)) V^T."""
    X, U, sig, V = _rand_X(48, 32, 0.1, 11)
    sched = svd_schedule(0.1)
    ws = []
    for st in sched:
        fn = qr_step if step == "qr" else chol_step
        X = fn(X, st["a"], st["b"], st["c"])
        ws.append((st["a"], st["b"], st["c"]))
        closed = planted_general(U, compose(sig, ws), V)
        assert np.linalg.norm(X - closed) / np.linalg.norm(closed) < 1e-13


def test_polar_invariant():
    """X_k^T A is symmetric positive semidefinite (X_k shares A's singular vectors)."""
    X0, U, sig, V = _rand_X(40, 25, 0.05, 2)
    X = X0.copy()
    for st in svd_schedule(0.05):
        X = qr_step(X, st["a"], st["b"], st["c"])
        M = X.T @ X0
        assert np.linalg.norm(M - M.T) < 1e-13 * np.linalg.norm(M)
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > -1e-13


def test_lanczos_interlacing_and_counts():
    A, lam = eig_uniform(400, 9)
    est = lanczos_slq(lambda v: A @ v, 400, seed=1)
    assert est["nodes"].max() <= lam.max() + 1e-12
    assert est["nodes"].min() >= lam.min() - 1e-12
    assert est["lmax"] >= lam.max() - 1e-10 and est["lmin"] <= lam.min() + 1e-10
    assert abs(est["weights"].sum() - est["nv"]) < 1e-10
    for t in [0.9, 0.5, 0.0]:
        true = int(np.sum(lam >= t))
        assert abs(count_above(est, t) - true) < 0.1 * 400


def _planted_eig_check(A, lam, fraction, which="largest", tol_val=1e-12, tol_res=1e-13, **kw):
    r = oracle.eig_partial(A, fraction=fraction, which=which, **kw)
    ex = np.sort(lam)[::-1] if which == "largest" else np.sort(lam)
    ex = ex[:r["k"]]
    met = oracle.eig_metrics(A, r["w"], r["V"], ex)
    assert met["value_rel_max"] < tol_val, met
    assert met["residual"] < tol_res, met
    assert met["orth"] < 1e-13 * math.sqrt(r["k"]) * 10, met
    return r, met


@pytest.mark.parametrize("n,f,seed", [(512, 0.1, 1000), (300, 0.2, 5), (257, 0.01, 6)])
def test_eig_planted_uniform(n, f, seed):
    A, lam = eig_uniform(n, seed)
    _planted_eig_check(A, lam, f)


def test_eig_planted_clusters_and_smallest():
    A, lam = eig_clustered(1024, 1002)
    r, _ = _planted_eig_check(A, lam, 0.2)
    r, _ = _planted_eig_check(A, lam, 0.01)
    # the smallest eigenvalues of the same matrix
    _planted_eig_check(A, lam, 0.05, which="smallest")


def test_eig_threshold_mode_negative_spectrum():
    """The paper's native problem (Algorithm 1): all negative eigenpairs."""
    g = rng(21)
    Q = haar(g, 200)
    lam = np.concatenate([-g.uniform(0.05, 1.0, 20), g.uniform(0.05, 3.0, 180)])
    A = planted_sym(Q, lam)
    r = oracle.eig_partial(A, tau=0.0, which="smallest")
    assert r["k"] == 20
    assert np.max(np.abs(r["w"] - np.sort(lam)[:20]) / np.abs(np.sort(lam)[:20])) < 1e-12


def test_eig_theorem1_and_containment():
    """Theorem 1: sin angle(V0, Q2) <= ||V0^T B||_2 / sigma_min(R11)."""
    g = rng(31)
    n = 256
    Q = haar(g, n)
    lam = g.uniform(-1, 1, n)
    A = planted_sym(Q, lam)
    r = oracle.eig_partial(A, fraction=0.1)
    V0 = Q[:, np.argsort(-lam)[:r["k"]]]
    B, Q2 = r["B"], r["Q2"]
    Qf, R = np.linalg.qr(B)
    ind = r["ind"]
    R11 = R[:ind - 1, :ind - 1]
    sin_angle = np.linalg.norm(V0 - Q2 @ (Q2.T @ V0), 2)
    bound = np.linalg.norm(V0.T @ B, 2) / np.linalg.svd(R11, compute_uv=False).min()
    assert sin_angle <= bound * (1 + 1e-6) + 1e-15
    assert sin_angle < 1e-12


def test_eig_band_prediction():
    """ell matches the count predicted by the scalar composite on the planted values."""
    A, lam = eig_uniform(600, 77)
    r = oracle.eig_partial(A, fraction=0.1)
    xs = (1 - 0.2) * (r["tau"] - lam) / r["mu"] - 0.2
    ws = [(st["a"], st["b"], st["c"]) for st in r["sched"]]
    pred = int(np.sum((compose(xs, ws) + 1) / 2 < 0.01))
    assert abs(r["ell"] - pred) <= max(3, 0.02 * pred)


@pytest.mark.parametrize("seed", range(6))
def test_eig_brute_force_jacobi(seed):
    g = rng(500 + seed)
    n = [12, 24, 40, 64, 33, 50][seed]
    G = g.standard_normal((n, n))
    A = 0.5 * (G + G.T)
    w_j, V_j = oracle.jacobi_eig(A)
    k = max(1, n // 5)
    r = oracle.eig_partial(A, k=k)
    scale = np.abs(w_j).max()
    assert np.max(np.abs(r["w"] - w_j[:k])) / scale < 1e-13
    # vectors up to sign (gaps of a Gaussian matrix are not tiny)
    d = np.abs(np.sum(r["V"] * V_j[:, :k], axis=0))
    assert np.max(np.abs(d - 1)) < 1e-9
    # smallest too
    r = oracle.eig_partial(A, k=k, which="smallest")
    assert np.max(np.abs(r["w"] - w_j[::-1][:k])) / scale < 1e-13


@pytest.mark.parametrize("seed", range(5))
def test_svd_brute_force_jacobi(seed):
    g = rng(700 + seed)
    m, n = [(20, 12), (40, 40), (64, 30), (30, 50), (64, 64)][seed]
    A = g.standard_normal((m, n))
    U_j, S_j, V_j = oracle.jacobi_svd(A if m >= n else A.T)
    if m < n:
        U_j, V_j = V_j, U_j
    k = max(1, min(m, n) // 5)
    r = oracle.svd_partial(A, k)
    assert np.max(np.abs(r["S"] - S_j[:k]) / S_j[:k]) < 1e-13
    dv = np.abs(np.sum(r["V"] * V_j[:, :k], axis=0))
    du = np.abs(np.sum(r["U"] * U_j[:, :k], axis=0))
    assert np.max(np.abs(dv - 1)) < 1e-9 and np.max(np.abs(du - 1)) < 1e-9


def test_jacobi_closed_forms():
    w, V = oracle.jacobi_eig(np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert np.allclose(w, [3.0, 1.0], atol=1e-15)
    assert np.allclose(np.abs(V), np.sqrt(0.5), atol=1e-15)
    w, V = oracle.jacobi_eig(np.diag([3.0, -1.0, 2.0]))
    assert np.array_equal(w, [3.0, 2.0, -1.0])
    U, S, V = oracle.jacobi_svd(np.array([[3.0, 0.0], [4.0, 5.0]]))
    assert np.allclose(S, [math.sqrt(45.0), math.sqrt(5.0)], atol=1e-14)


@pytest.mark.parametrize("m,n,k,maker", [(1024, 1024, 51, "geo"), (600, 300, 30, "log"),
                                         (300, 600, 30, "log")])
def test_svd_planted(m, n, k, maker):
    if maker == "geo":
        A, sig = svd_geometric(m, n, 1001)
    else:
        A, sig = svd_loguniform(max(m, n), min(m, n), 1003)
        if m < n:
            A = A.T.copy()
    r = oracle.svd_partial(A, k)
    met = oracle.svd_metrics(A, r["U"], r["S"], r["V"], sig[:k])
    assert met["value_rel_max"] < 1e-12, met
    assert met["residual"] < 1e-13, met
    assert max(met["orth_u"], met["orth_v"]) < 1e-12, met


def test_svd_threshold_percent(golden):
    """Sec. 7.2/7.4: with D[i] = 0.5^(100 i/N), thresholds s = 0.1 .. 1e-4 select
    3/7/10/13 % of the singular values (threshold mode of Algorithm 2)."""
    f = golden["svd_threshold_to_percent"]
    N = 400
    g = rng(55)
    U, V = haar(g, N), haar(g, N)
    D = 0.5 ** (100.0 * np.arange(N) / N)
    A = planted_general(U, D, V)
    for s, pct in zip(f["s"], f["percent"]):
        r = oracle.svd_partial(A, s=s, replay={"alpha": 1.0})
        assert abs(100.0 * r["k"] / N - pct) <= 0.5, (s, r["k"])
        assert r["k"] == int(np.sum(D >= s))
        assert np.max(np.abs(r["S"] - D[:r["k"]]) / D[:r["k"]]) < 1e-12


def test_replay_reproduces_auto():
    A, lam = eig_uniform(256, 4)
    r1 = oracle.eig_partial(A, fraction=0.15)
    rep = dict(tau=r1["tau"], mu=r1["mu"], rho=r1["rho"], kinds=[s["kind"] for s in r1["sched"]])
    r2 = oracle.eig_partial(A, fraction=0.15, replay=rep)
    assert np.array_equal(r1["w"], r2["w"]) and r1["ell"] == r2["ell"]


def test_edge_cases():
    # everything wanted
    A, lam = eig_uniform(40, 8)
    r = oracle.eig_partial(A, fraction=1.0)
    assert r["k"] == 40 and np.max(np.abs(r["w"] - np.sort(lam)[::-1])) < 1e-13
    # tiny n
    r = oracle.eig_partial(np.array([[2.0, 1.0], [1.0, 2.0]]), k=1)
    assert abs(r["w"][0] - 3.0) < 1e-14
    # multiple eigenvalue: top-3 of diag(5,5,5,1,...) any basis of the eigenspace
    g = rng(9)
    Q = haar(g, 30)
    lam = np.concatenate([[5.0, 5.0, 5.0], g.uniform(-1, 1, 27)])
    A = planted_sym(Q, lam)
    r = oracle.eig_partial(A, k=3)
    assert np.max(np.abs(r["w"] - 5.0)) < 1e-13
    P = r["V"] @ r["V"].T
    P0 = Q[:, :3] @ Q[:, :3].T
    assert np.linalg.norm(P - P0) < 1e-12
    # ragged SVD shapes
    A = rng(10).standard_normal((37, 23))
    r = oracle.svd_partial(A, 5)
    assert np.allclose(r["S"], np.linalg.svd(A, compute_uv=False)[:5], rtol=1e-13)


def test_svd_cut_is_relative_for_graded_spectra():
    """Nodes of A^T A span many decades for ill-conditioned A: a node counts as
    distinct on a relative scale, and without a lower node the cut is half
    the node (never 0, which would map every singular value to 1)."""
    from oracle.estimator import _cut_below, choose_svd_threshold
    est = dict(n=100, nv=1, lmax=1.0, lmin=-1e-3,
               nodes=np.array([1.0, 1e-3, 5e-7, 1e-9]), weights=np.array([0.1, 0.2, 0.3, 0.4]))
    # the count reaches kt = 50 at the node 5e-7
    assert _cut_below(est, 50) is None                       # absolute rule: nothing distinct below
    assert _cut_below(est, 50, nonneg=True) == pytest.approx(0.5 * (5e-7 + 1e-9))
    est2 = dict(est, nodes=np.array([1.0, 1e-3, 5e-7, 5e-7 * (1 - 1e-9)]))
    assert _cut_below(est2, 50, nonneg=True) == pytest.approx(2.5e-7)
    alpha, s = choose_svd_threshold(est, 40)
    assert s > 1e-6 and alpha == 1.0


def test_svd_graded_kappa_1e12_keeps_ell_below_n():
    """A geometric spectrum down to 1e-12 with ~19% wanted: ell < n and the
    top-k values are exact."""
    from synthetic import svd_geometric
    import oracle
    A, sig = svd_geometric(256, 256, 4041, kappa=9.6e11)
    k = 49
    r = oracle.svd_partial(A, k=k)
    assert r["ell"] < 256
    assert np.max(np.abs(r["S"] - sig[:k]) / sig[:k]) <= 1e-12


def test_cost_policy_turns_qr_steps_into_cholesky_steps():
    """A clustered spectrum with 1% wanted: the plain cut lands in the top
    clusters, rho is large and QR-based steps follow; the cost policy picks a
    lower cut whose three Cholesky-based steps and larger subspace cost fewer
    Table 1 flops, with the same planted values."""
    from oracle.estimator import predicted_flops
    A, lam = eig_clustered(1024, 1002)
    rp = oracle.eig_partial(A, fraction=0.01, tau_policy="plain")
    rc = oracle.eig_partial(A, fraction=0.01, tau_policy="cost")
    assert "qr" in [st["kind"] for st in rp["sched"]]
    assert [st["kind"] for st in rc["sched"]] == ["chol"] * 3
    assert rc["tau"] < rp["tau"] and rc["ell"] > rp["ell"]
    assert predicted_flops(rc["sched"], 1024, rc["ell"]) < predicted_flops(rp["sched"], 1024, rp["ell"])
    ex = np.sort(lam)[::-1][:rc["k"]]
    for r in (rp, rc):
        met = oracle.eig_metrics(A, r["w"], r["V"], ex)
        assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13, met
    # the band edge predicts the subspace size (the count of planted values
    # above it) to within the non-rank-revealing slack of the plain QR
    from oracle.estimator import _band_edge
    edge = rc["tau"] - rc["mu"] * (_band_edge(rc["sched"], 0.2, 0.01) + 0.2) / 0.8
    pred = int(np.sum(lam >= edge))
    assert abs(rc["ell"] - pred) <= max(3, 0.02 * pred)


def test_omega_qr_gives_the_same_subspace_values():
    """QR of B Omega (Sec. 4.1, randomised rank-revealing form): same planted
    values, a subspace containing the wanted one."""
    A, lam = eig_uniform(400, 61)
    r = oracle.eig_partial(A, fraction=0.1, use_omega=True)
    ex = np.sort(lam)[::-1][:r["k"]]
    met = oracle.eig_metrics(A, r["w"], r["V"], ex)
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13, met
