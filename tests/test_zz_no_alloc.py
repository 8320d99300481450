"""qdwhp_eig_noalloc (the solve with the library's fixed workspace array)
against qdwhp_eig (caller workspace) through the C ABI: bitwise equal
results on two calls in a row, the second with a smaller input; values
against the planted spectrum; an oversized problem is rejected."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call(q, torch, fn, A, f, with_ws):
    n = A.shape[0]
    k = min(n, max(1, int(np.floor(f * n + 0.5))))
    o = q.default_opts()
    w = torch.empty(k, dtype=torch.float64, device=A.device)
    Vb = torch.empty((k, n), dtype=torch.float64, device=A.device)
    info = q.Info()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    L = q.lib()
    if with_ws:
        nb = L.qdwhp_eig_workspace(n, f, ctypes.byref(o))
        ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=A.device)
        r = L.qdwhp_eig(p(A), n, n, f, q.LARGEST, p(w), p(Vb), n, p(ws), nb, ctypes.byref(o), st,
                        ctypes.byref(info))
    else:
        r = L.qdwhp_eig_noalloc(p(A), n, n, f, q.LARGEST, p(w), p(Vb), n, ctypes.byref(o), st,
                                ctypes.byref(info))
    torch.cuda.synchronize()
    return r, w, Vb, info


def test_noalloc_equals_workspace_entry_point():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_14186_amd as q
    from synthetic import eig_uniform, eig_clustered
    cases = [(eig_clustered, 1000, 0.2, 11), (eig_uniform, 600, 0.1, 12)]   # second call smaller
    for make, n, f, seed in cases:
        A, lam = make(n, seed, device=torch.device("cuda"))
        A = A.contiguous()
        print(f"noalloc n={n} f={f}", flush=True)
        r0, w0, V0, i0 = _call(q, torch, None, A, f, True)
        r1, w1, V1, i1 = _call(q, torch, None, A, f, False)
        assert r0 == 0 and r1 == 0
        assert bool((w0 == w1).all()) and bool((V0 == V1).all())
        assert i1.ell == i0.ell and i1.k == i0.k
        exact = np.sort(lam)[::-1][:len(w1)]
        assert np.max(np.abs(w1.cpu().numpy() - exact) / np.abs(exact)) <= 1e-12


def test_noalloc_rejects_problems_beyond_its_array():
    import torch
    import paper_2104_14186_amd as q
    L = q.lib()
    o = q.default_opts()
    cap = L.qdwhp_noalloc_max_bytes()
    n = 16
    while L.qdwhp_eig_workspace(n, 0.1, ctypes.byref(o)) <= cap:
        n *= 2
    print(f"noalloc limit: n={n} needs {L.qdwhp_eig_workspace(n, 0.1, ctypes.byref(o))} > {cap}", flush=True)
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    w = torch.empty(1, dtype=torch.float64, device="cuda")
    V = torch.empty((1, n), dtype=torch.float64, device="cuda")
    info = q.Info()
    st = L.qdwhp_eig_noalloc(ctypes.c_void_p(A.data_ptr()), n, n, 0.1, q.LARGEST, ctypes.c_void_p(w.data_ptr()),
                             ctypes.c_void_p(V.data_ptr()), n, ctypes.byref(o),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(info))
    assert st == 4 and info.status == 4
