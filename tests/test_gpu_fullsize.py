"""Parity at the benchmark sizes, in the configuration bench.py times.

The oracle cannot run at these sizes in seconds, so each case checks what the
construction fixes exactly: the computed values against the planted spectrum
(relative error <= 1e-12) and, on sampled vectors, residuals against ||A||_2
(<= 1e-13) and orthogonality.  The mixed-precision case checks its values at
the same bar and reports its (FP32-level) vector residuals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _sample(k, cnt=16):
    return np.unique(np.linspace(0, k - 1, min(k, cnt)).round().astype(int))


def _eig_check(torch, A, w, V, exact, norm):
    k = len(w)
    rel = np.max(np.abs(w.cpu().numpy() - exact[:k]) / np.abs(exact[:k]))
    idx = torch.as_tensor(_sample(k), device=w.device)
    Vs = V[:, idx].contiguous()
    R = A @ Vs - Vs * w[idx][None, :]
    res = float(R.norm(dim=0).max()) / norm
    orth = float((Vs.t() @ Vs - torch.eye(len(idx), dtype=Vs.dtype, device=Vs.device)).abs().max())
    return rel, res, orth


def _svd_check(torch, A, U, S, V, exact):
    k = len(S)
    rel = np.max(np.abs(S.cpu().numpy() - exact[:k]) / exact[:k])
    idx = torch.as_tensor(_sample(k), device=S.device)
    Us, Vs, Ss = U[:, idx].contiguous(), V[:, idx].contiguous(), S[idx]
    r1 = (A @ Vs - Us * Ss[None, :]).norm(dim=0).max()
    r2 = (A.t() @ Us - Vs * Ss[None, :]).norm(dim=0).max()
    res = float(max(r1, r2)) / float(exact[0])
    eye = torch.eye(len(idx), dtype=Us.dtype, device=Us.device)
    orth = float(max((Us.t() @ Us - eye).abs().max(), (Vs.t() @ Vs - eye).abs().max()))
    return rel, res, orth


@pytest.mark.parametrize("fraction", [0.2, 0.01])
def test_eig16384_clustered(fraction):
    torch = _torch()
    import paper_2104_14186_amd as q
    from synthetic import eig_clustered, CONFIG_SEEDS
    print("eig16384 clustered", fraction, flush=True)
    A, lam = eig_clustered(16384, CONFIG_SEEDS["eig16384"], device=torch.device("cuda"))
    w, V, info = q.eig(A, fraction=fraction, return_info=True)
    torch.cuda.synchronize()
    exact = np.sort(lam)[::-1]
    rel, res, orth = _eig_check(torch, A, w, V, exact, float(np.max(np.abs(lam))))
    print(f"  k={len(w)} ell={info['ell']} kinds={info['kinds']} rel={rel:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
    assert len(w) == int(np.floor(fraction * 16384 + 0.5))
    assert rel <= 1e-12 and res <= 1e-13 and orth <= 1e-12


def test_svd4096_kappa1e16_top5():
    torch = _torch()
    import paper_2104_14186_amd as q
    from synthetic import svd_geometric, CONFIG_SEEDS
    print("svd4096 kappa 1e16 top 5%", flush=True)
    A, sig = svd_geometric(4096, 4096, CONFIG_SEEDS["svd4096"], kappa=1e16, device=torch.device("cuda"))
    U, S, V, info = q.svd(A, 205, return_info=True)
    torch.cuda.synchronize()
    rel, res, orth = _svd_check(torch, A, U, S, V, np.asarray(sig))
    print(f"  ell={info['ell']} kinds={info['kinds']} rel={rel:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
    assert info["kinds"][0] == "qr"
    assert rel <= 1e-12 and res <= 1e-13 and orth <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_svd16384x8192_loguniform_top10(precision):
    torch = _torch()
    import paper_2104_14186_amd as q
    from synthetic import svd_loguniform, CONFIG_SEEDS
    print("svd16384x8192 top 10% precision", precision, flush=True)
    A, sig = svd_loguniform(16384, 8192, CONFIG_SEEDS["svd16384x8192"], device=torch.device("cuda"))
    U, S, V, info = q.svd(A, 819, opts=q.default_opts(precision=precision), return_info=True)
    torch.cuda.synchronize()
    rel, res, orth = _svd_check(torch, A, U, S, V, np.asarray(sig))
    print(f"  ell={info['ell']} kinds={info['kinds']} rel={rel:.2e} res={res:.2e} orth={orth:.2e} "
          f"ms={info['ms'][7]:.0f}", flush=True)
    assert rel <= 1e-12
    if precision == 0:
        assert res <= 1e-13 and orth <= 1e-12
    else:   # vectors carry the FP32 rounding of the low-precision products
        assert res <= 1e-5 and orth <= 1e-5
