"""Kernel-level parity of the HIP building blocks against FP64 host references.

Each case prints its shape before the GPU call so a failing case is named."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _cm(torch, X):
    """Column-major device buffer of host matrix X (shape (cols, rows))."""
    return torch.from_numpy(np.ascontiguousarray(X.T)).cuda()


def _host(T):
    return T.cpu().numpy().T


@pytest.mark.parametrize("m,n,k,ta,tb", [
    (128, 128, 16, 0, 0), (300, 257, 129, 0, 0), (257, 300, 77, 1, 0),
    (190, 64, 300, 0, 1), (1, 1, 1, 1, 1), (513, 511, 1000, 1, 1), (5, 700, 3, 0, 0)])
def test_dgemm_parity(m, n, k, ta, tb):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(m * 7 + n + k)
    A = g.standard_normal((k, m) if ta else (m, k))
    B = g.standard_normal((n, k) if tb else (k, n))
    C = g.standard_normal((m, n))
    print(f"dgemm m={m} n={n} k={k} ta={ta} tb={tb}", flush=True)
    Cd = _cm(torch, C)
    q.dgemm(_cm(torch, A), _cm(torch, B), Cd, alpha=0.75, beta=-0.5, transa=ta, transb=tb)
    torch.cuda.synchronize()
    ref = 0.75 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C
    err = np.abs(_host(Cd) - ref).max() / (np.abs(ref).max() + 1e-300)
    assert err < 1e-14 * max(1, np.sqrt(k)), err


def test_dgemm_upper_tiles_only():
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(3)
    n, k = 400, 150
    X = g.standard_normal((k, n))
    print("dgemm upper n=400", flush=True)
    C = np.full((n, n), 7.0)
    Cd = _cm(torch, C)
    q.dgemm(_cm(torch, X), _cm(torch, X), Cd, transa=True, upper=True)
    torch.cuda.synchronize()
    got = _host(Cd)
    ref = X.T @ X
    iu = np.triu_indices(n)
    assert np.abs(got[iu] - ref[iu]).max() < 1e-12
    # a strictly-lower tile far from the diagonal is untouched
    assert np.all(got[300:, :100] == 7.0)


# 129..159: the recursion's first half needs a bigger product buffer one
# level down than the top split does (the workspace covers every level)
@pytest.mark.parametrize("n", [1, 63, 64, 65, 129, 140, 159, 200, 517])
def test_spd_inverse(n):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(n)
    X = g.standard_normal((n + 5, n))
    Z = np.eye(n) + 3.0 * X.T @ X / n
    print(f"spd_inverse n={n}", flush=True)
    Zi = q.spd_inverse(torch.from_numpy(Z).cuda()).cpu().numpy()
    ref = np.linalg.inv(Z)
    assert np.abs(Zi - ref).max() / np.abs(ref).max() < 1e-13 * np.linalg.cond(Z)


@pytest.mark.parametrize("m,n", [(1, 1), (40, 40), (300, 129), (513, 256), (1024, 512), (700, 700),
                                 (1000, 385)])
def test_qr(m, n):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(m + n)
    A = g.standard_normal((m, n))
    print(f"qr m={m} n={n}", flush=True)
    Q, R, tau = q.qr(torch.from_numpy(A).cuda())
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.abs(Q @ R - A).max() < 2e-15 * np.abs(A).max() * np.sqrt(m)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 2e-15 * np.sqrt(m)
    Rl = np.linalg.qr(A, mode="r")
    assert np.abs(np.abs(np.diag(R)) - np.abs(np.diag(Rl))).max() < 1e-12 * np.abs(Rl).max()


def _qr_path(q, torch, A, recon):
    old = q.tune_get("qr.recon", 1)
    q.tune_set("qr.recon", recon)
    try:
        Q, R, tau = q.qr(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
    finally:
        q.tune_set("qr.recon", old)
    return Q.cpu().numpy(), R.cpu().numpy(), tau.cpu().numpy()



@pytest.mark.parametrize("m,n", [(3000, 1000), (1500, 1500), (4100, 193)])
def test_qr_overlapped_trailing_updates(m, n):
    """The trailing updates on a helper stream, overlapping the next
    panel's factorization, give the one-stream factorization to rounding
    (only the K split of the narrow product differs)."""
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(m + 3 * n)
    A = g.standard_normal((m, n)) * np.geomspace(1.0, 1e-3, n)[None, :]
    print(f"qr overlap m={m} n={n}", flush=True)
    old = q.tune_get("qr.overlap", 1)
    out = {}
    try:
        for ov in (0, 1):
            q.tune_set("qr.overlap", ov)
            out[ov] = _qr_path(q, torch, A, 1)
    finally:
        q.tune_set("qr.overlap", old)
    (Q0, R0, t0), (Q1, R1, t1) = out[0], out[1]
    sc = np.abs(A).max()
    assert np.abs(Q1 @ R1 - A).max() / sc < 4e-15 * np.sqrt(m)
    assert np.abs(Q1.T @ Q1 - np.eye(n)).max() < 4e-15 * np.sqrt(m)
    assert np.abs(R1 - R0).max() < 1e-12 * sc * np.sqrt(m)
    assert np.abs(t1 - t0).max() < 1e-12
    assert np.abs(Q1 - Q0).max() < 1e-11

@pytest.mark.parametrize("m,n,kind", [(2000, 300, "gauss"), (517, 517, "gauss"), (3000, 700, "graded"),
                                      (1200, 400, "dependent"), (800, 800, "projector")])
def test_qr_reconstructed_panels_match_column_steps(m, n, kind):
    """Sub-panels by Cholesky QR with Householder reconstruction give the
    LAPACK-convention Householder factorization of the column steps (same
    R, reflectors and tau to rounding); panels that fail the checks (exactly
    dependent columns, the projector's rank drop) are restored and redone by
    the column steps."""
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(m + 7 * n)
    A = g.standard_normal((m, n))
    if kind == "graded":
        A = A * np.geomspace(1.0, 1e-4, n)[None, :]
    elif kind == "dependent":
        A[:, 200:230] = A[:, 10:40] @ g.standard_normal((30, 30))     # rank drop inside a panel
    elif kind == "projector":
        Qh, _ = np.linalg.qr(g.standard_normal((n, n)))
        d = np.concatenate([np.ones(n - 150), np.geomspace(0.3, 1e-15, 150)])
        A = (Qh * d) @ Qh.T
    print(f"qr recon vs column steps m={m} n={n} {kind}", flush=True)
    Q1, R1, t1 = _qr_path(q, torch, A, 1)
    Q0, R0, t0 = _qr_path(q, torch, A, 0)
    sc = np.abs(A).max()
    for name, Q, R in (("reconstructed", Q1, R1), ("column steps", Q0, R0)):
        res, orth = np.abs(Q @ R - A).max() / sc, np.abs(Q.T @ Q - np.eye(n)).max()
        print(f"  {name}: residual {res:.2e} orthogonality {orth:.2e}", flush=True)
        assert res < 4e-15 * np.sqrt(m)
        assert orth < 4e-15 * np.sqrt(m)
    if kind in ("gauss", "graded"):
        # full rank: the two factorizations agree entry by entry, up to the
        # sign of the last row of a square matrix (the column steps keep
        # R(n,n) with tau = 0 there, the reconstruction reflects it, tau = 2:
        # both are Householder factorizations)
        D = np.sign(np.diag(R1)) * np.sign(np.diag(R0))
        flips = np.nonzero(D < 0)[0]
        assert len(flips) == 0 or (m == n and list(flips) == [n - 1])
        assert np.abs(D[:, None] * R1 - R0).max() < 1e-12 * sc * np.sqrt(m)
        assert np.abs(t1[D > 0] - t0[D > 0]).max() < 1e-12
        assert np.abs(Q1 * D[None, :] - Q0).max() < 1e-11
    else:
        # rank drop: |R_ii| agree up to the first rounding-level one (after
        # it the reflectors of the dependent columns are rounding noise and
        # the later R_ii are not determined by A)
        d1, d0 = np.abs(np.diag(R1)), np.abs(np.diag(R0))
        first = int(np.argmax(d0 < 1e-8 * sc))
        assert first > 0 and d1[first] < 1e-8 * sc
        assert np.abs(d1[:first] - d0[:first]).max() < 1e-12 * sc * np.sqrt(m)


@pytest.mark.parametrize("n,c0", [(300, 170), (700, 300)])
def test_qr_trailing_columns(n, c0):
    """Columns c0.. of Q of a square matrix (the Q2 of the projector)."""
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(11)
    A = g.standard_normal((n, n))
    print("qr trailing columns", flush=True)
    Qc, R, _ = q.qr(torch.from_numpy(A).cuda(), c0=c0, q=n - c0)
    Qf, _ = np.linalg.qr(A)
    P1 = Qc.cpu().numpy() @ Qc.cpu().numpy().T
    P2 = Qf[:, c0:] @ Qf[:, c0:].T
    assert np.abs(P1 - P2).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 100, 257])
def test_syev(n):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(n + 3)
    G = g.standard_normal((n, n))
    H = 0.5 * (G + G.T)
    print(f"syev n={n}", flush=True)
    w, W, sw = q.syev(torch.from_numpy(H).cuda())
    w, W = w.cpu().numpy(), W.cpu().numpy()
    ref = np.sort(np.linalg.eigvalsh(H))[::-1]
    sc = np.abs(ref).max()
    assert np.abs(w - ref).max() < 5e-15 * sc * max(1, np.sqrt(n))
    assert np.abs(H @ W - W * w[None, :]).max() < 5e-15 * sc * max(1, np.sqrt(n))
    assert np.abs(W.T @ W - np.eye(n)).max() < 5e-15 * max(1, np.sqrt(n))


@pytest.mark.parametrize("n", [100, 333])
def test_syev_helper_stream_path_matches_single_launch_rounds(n):
    """Above the fused size the eigenvector update of each round runs on a
    helper stream from a ring of rotation slots; it applies the same
    arithmetic as the one-launch round, so the results are identical."""
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(n + 11)
    G = g.standard_normal((n, n))
    H = torch.from_numpy(0.5 * (G + G.T)).cuda()
    print(f"syev streams n={n}", flush=True)
    out = []
    old = q.tune_get("jacobi.fused_max", 2048)
    try:
        for thr in (1 << 40, 0, 0):   # fused, then the helper-stream path twice
            q.tune_set("jacobi.fused_max", thr)
            w, W, sw = q.syev(H)
            torch.cuda.synchronize()
            out.append((w.clone(), W.clone(), sw))
    finally:
        q.tune_set("jacobi.fused_max", old)
    for w, W, sw in out[1:]:
        assert sw == out[0][2]
        assert bool((w == out[0][0]).all()) and bool((W == out[0][1]).all())


@pytest.mark.parametrize("n", [1, 2, 32, 45, 200])
def test_gesvj(n):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(n + 5)
    R = np.triu(g.standard_normal((n, n)))
    print(f"gesvj n={n}", flush=True)
    U, S, V, sw = q.gesvj(torch.from_numpy(R).cuda())
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.svd(R, compute_uv=False)
    assert np.abs(S - ref).max() < 5e-15 * ref.max() * max(1, np.sqrt(n))
    assert np.abs(R @ V - U * S[None, :]).max() < 5e-15 * ref.max() * max(1, np.sqrt(n))
    assert np.abs(V.T @ V - np.eye(n)).max() < 5e-15 * max(1, np.sqrt(n))


@pytest.mark.parametrize("m,n,k,ta,tb,upper", [
    (300, 257, 129, 0, 0, 0), (257, 300, 77, 1, 0, 0), (190, 64, 300, 0, 1, 0),
    (513, 511, 100, 1, 1, 0), (333, 333, 200, 1, 0, 1)])
def test_dgemm_tile_size_does_not_change_results(m, n, k, ta, tb, upper):
    """64x64 and 128x128 tiles sum every element in the same k order."""
    torch = _torch()
    import paper_2104_14186_amd as q
    print("tiles", m, n, k, ta, tb, upper, flush=True)
    g = np.random.default_rng(9)
    A = g.standard_normal((k, m) if ta else (m, k))
    B = g.standard_normal((n, k) if tb else (k, n))
    dA, dB = _cm(torch, A), _cm(torch, B)
    out = []
    old = q.tune_get("gemm.small_tiles", 96)
    try:
        for thr in (0, 1 << 40):
            q.tune_set("gemm.small_tiles", thr)
            C = torch.zeros((n, m), dtype=torch.float64, device="cuda")
            q.dgemm(dA, dB, C, 1.0, 0.0, transa=bool(ta), transb=bool(tb), upper=bool(upper))
            torch.cuda.synchronize()
            out.append(C.clone())
    finally:
        q.tune_set("gemm.small_tiles", old)
    if upper:   # only the upper triangle is defined for an upper-tile output
        out = [torch.triu(c.t()) for c in out]
    assert bool((out[0] == out[1]).all())


@pytest.mark.parametrize("n,leaf", [(700, 256), (1100, 300)])
def test_syev_dc_side_by_side_bitwise(n, leaf):
    """The two sides of a split (bases, blocks, leaf Jacobi solves) run side
    by side on two streams from two host threads, or one after the other
    ("dc.concurrent" = 0): the same kernels on the same data, so the
    results are bitwise equal."""
    torch = _torch()
    import paper_2104_14186_amd as q
    from synthetic import eig_uniform
    A, lam = eig_uniform(n, 950 + n)
    print(f"syev_dc side by side n={n} leaf={leaf}", flush=True)
    old = (q.tune_get("dc.leaf", 512), q.tune_get("dc.concurrent", 1))
    out = {}
    try:
        q.tune_set("dc.leaf", leaf)
        for cc in (0, 1):
            q.tune_set("dc.concurrent", cc)
            w, W, depth = q.syev_dc(torch.from_numpy(A).cuda())
            torch.cuda.synchronize()
            out[cc] = (w.cpu().numpy(), W.cpu().numpy(), depth)
    finally:
        q.tune_set("dc.leaf", old[0])
        q.tune_set("dc.concurrent", old[1])
    assert out[0][2] >= 1 and out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    ex = np.sort(lam)[::-1]
    assert np.max(np.abs(out[1][0] - ex)) / np.abs(lam).max() < 1e-13


@pytest.mark.parametrize("n,spec,leaf", [(300, "uniform", 64), (1000, "uniform", 128), (1500, "clustered", 256),
                                         (700, "median_cluster", 128), (900, "uniform", 4096)])
def test_syev_dc(n, spec, leaf):
    """Full spectrum by QDWH-based spectral divide and conquer (Sec. 3.2):
    planted eigenvalues, residual and orthogonality of every eigenvector;
    a spectrum with a tight cluster at the median makes a split fail its
    check and fall back to Jacobi on that block."""
    torch = _torch()
    import paper_2104_14186_amd as q
    from synthetic import eig_uniform, eig_clustered, rng, haar, planted_sym
    if spec == "uniform":
        A, lam = eig_uniform(n, 900 + n)
    elif spec == "clustered":
        A, lam = eig_clustered(n, 901)
    else:
        g = rng(902)
        Q = haar(g, n)
        lam = np.concatenate([g.uniform(-1, 1, n // 2), 0.1 + 1e-13 * g.uniform(-1, 1, n - n // 2)])
        A = planted_sym(Q, lam)
    print(f"syev_dc n={n} {spec} leaf={leaf}", flush=True)
    old = q.tune_get("dc.leaf", 512)
    try:
        q.tune_set("dc.leaf", leaf)
        w, W, depth = q.syev_dc(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
    finally:
        q.tune_set("dc.leaf", old)
    w, W = w.cpu().numpy(), W.cpu().numpy()
    print(f"  depth {depth}", flush=True)
    ex = np.sort(lam)[::-1]
    scale = np.abs(lam).max()
    assert np.max(np.abs(w - ex)) / scale < 1e-13
    R = A @ W - W * w[None, :]
    assert np.linalg.norm(R, axis=0).max() / scale < 1e-13
    assert np.abs(W.T @ W - np.eye(n)).max() < 1e-12
    if leaf < n and spec != "median_cluster":
        assert depth >= 1
