"""Mixed precision (FP32 matrix cores inside the Cholesky-based steps, FP64
polish) against the FP64 oracle: values to the FP64 bar, vectors to FP32 level."""
import numpy as np
import pytest

import oracle
from synthetic import eig_uniform, svd_loguniform, svd_geometric

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_14186_amd as q
    return torch, q


@pytest.mark.parametrize("m,n,k,ta,tb", [(300, 257, 129, 0, 0), (257, 300, 77, 1, 0), (400, 400, 1000, 0, 1)])
def test_gemm_f32(m, n, k, ta, tb):
    torch, q = _gpu()
    g = np.random.default_rng(m + k)
    A = g.standard_normal((k, m) if ta else (m, k))
    B = g.standard_normal((n, k) if tb else (k, n))
    C = g.standard_normal((m, n))
    print(f"gemm f32 m={m} n={n} k={k}", flush=True)
    cm = lambda X: torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    Cd = cm(C)
    q.dgemm(cm(A), cm(B), Cd, alpha=0.5, beta=2.0, transa=ta, transb=tb, f32=True)
    torch.cuda.synchronize()
    ref = 0.5 * ((A.T if ta else A) @ (B.T if tb else B)) + 2.0 * C
    got = Cd.cpu().numpy().T
    scale = 0.5 * np.abs(A).max() * np.abs(B).max() * k
    err = np.abs(got - ref).max() / scale
    assert err < 1e-6, err
    assert err > 1e-13   # the FP32 path really rounds


def test_eig_mixed_values():
    torch, q = _gpu()
    A, lam = eig_uniform(512, 1000)
    o = q.default_opts(precision=q.MIXED_FP32, tol=0.05)
    print("eig mixed n=512", flush=True)
    w, V, info = q.eig(torch.from_numpy(A).cuda(), fraction=0.1, opts=o, return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    r = oracle.eig_partial(A, fraction=0.1, tol=0.05)
    exact = np.sort(lam)[::-1][:len(w)]
    assert np.max(np.abs(w - r["w"]) / np.abs(r["w"])) < 1e-12
    assert np.max(np.abs(w - exact) / np.abs(exact)) < 1e-12
    met = oracle.eig_metrics(A, w, V)
    print("mixed eig residual", met["residual"], "orth", met["orth"])
    assert met["residual"] < 1e-5 and met["orth"] < 1e-10


@pytest.mark.parametrize("m,n,k,kind", [(600, 300, 30, "log"), (512, 512, 26, "geo")])
def test_svd_mixed_values(m, n, k, kind):
    torch, q = _gpu()
    if kind == "log":
        A, sig = svd_loguniform(m, n, 1003)
    else:
        A, sig = svd_geometric(m, n, 1001)
    o = q.default_opts(precision=q.MIXED_FP32, tol=0.05)
    print(f"svd mixed {m}x{n}", flush=True)
    U, S, V, info = q.svd(torch.from_numpy(A).cuda(), k, opts=o, return_info=True)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    r = oracle.svd_partial(A, k, tol=0.05)
    assert np.max(np.abs(S - r["S"]) / r["S"]) < 1e-12
    assert np.max(np.abs(S - sig[:k]) / sig[:k]) < 1e-12
    met = oracle.svd_metrics(A, U, S, V)
    print("mixed svd residual", met["residual"])
    assert met["residual"] < 1e-5
