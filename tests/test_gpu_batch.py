"""Ragged batches, the persistent grouped GEMM and the request server.

Batched and served results must equal standalone calls bitwise (same kernels,
launch shapes independent of the batch or mix); values are also checked
against the planted spectra.  Each case prints its shapes before GPU work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _specs(torch):
    from synthetic import eig_uniform, svd_geometric, eig_clustered
    dev = torch.device("cuda")
    specs, exact = [], []
    for n, f, seed in [(256, 0.1, 11), (130, 0.2, 12), (384, 0.05, 13)]:
        A, lam = eig_uniform(n, seed, device=dev)
        specs.append(dict(type="eig", A=A, fraction=f))
        exact.append(np.sort(lam)[::-1])
    A, lam = eig_clustered(300, 14, device=dev)
    specs.append(dict(type="eig", A=A, fraction=0.1, which="smallest"))
    exact.append(np.sort(lam))
    for m, n, k, seed in [(300, 200, 10, 15), (256, 256, 25, 16), (150, 320, 12, 17)]:
        if m >= n:
            A, s = svd_geometric(m, n, seed, kappa=1e10, device=dev)
        else:   # wide: transpose of a tall planted matrix
            A, s = svd_geometric(n, m, seed, kappa=1e10, device=dev)
            A = A.t().contiguous()
        specs.append(dict(type="svd", A=A, k=k))
        exact.append(np.asarray(s))
    return specs, exact


def _standalone(q, sp):
    if sp["type"] == "eig":
        return q.eig(sp["A"], fraction=sp["fraction"], which=sp.get("which", "largest"))
    return q.svd(sp["A"], sp["k"])


def _same(a, b):
    return all(bool((x == y).all()) for x, y in zip(a, b))


@pytest.mark.parametrize("transa,transb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_grouped_gemm_matches_host_and_single_launches(transa, transb):
    torch = _torch()
    import paper_2104_14186_amd as q
    g = np.random.default_rng(5)
    shapes = [(300, 257, 129), (1, 1, 1), (128, 128, 16), (5, 700, 3), (513, 130, 200), (64, 0, 5),
              (200, 100, 0)] + [(int(g.integers(1, 260)), int(g.integers(1, 260)), int(g.integers(1, 260)))
                               for _ in range(30)]
    print("grouped", transa, transb, len(shapes), flush=True)
    As, Bs, Cs, Cs1, ref, al, be = [], [], [], [], [], [], []
    for (m, n, k) in shapes:
        A = g.standard_normal((k, m) if transa else (m, k))
        B = g.standard_normal((n, k) if transb else (k, n))
        C = g.standard_normal((m, n))
        a, b = float(g.uniform(-2, 2)), float(g.uniform(-1, 1))
        opA = A.T if transa else A
        opB = B.T if transb else B
        ref.append(a * opA @ opB + b * C)
        As.append(torch.from_numpy(np.ascontiguousarray(A.T)).cuda())
        Bs.append(torch.from_numpy(np.ascontiguousarray(B.T)).cuda())
        Cs.append(torch.from_numpy(np.ascontiguousarray(C.T)).cuda())
        Cs1.append(Cs[-1].clone())
        al.append(a); be.append(b)
    q.dgemm_grouped(As, Bs, Cs, al, be, transa=bool(transa), transb=bool(transb))
    for i, (m, n, k) in enumerate(shapes):
        if min(m, n, k) > 0:
            q.dgemm(As[i], Bs[i], Cs1[i], al[i], be[i], transa=bool(transa), transb=bool(transb))
    torch.cuda.synchronize()
    for i, (m, n, k) in enumerate(shapes):
        got = Cs[i].cpu().numpy().T
        if got.size == 0:
            continue
        scale = max(1.0, np.abs(ref[i]).max()) * np.sqrt(max(k, 1))
        assert np.abs(got - ref[i]).max() <= 4e-15 * scale, (i, m, n, k)
        if min(m, n, k) > 0:
            assert bool((Cs[i] == Cs1[i]).all()), ("grouped differs from single launch", i, m, n, k)


@pytest.mark.parametrize("lanes", [1, 4])
def test_batched_equals_standalone_bitwise(lanes):
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = _specs(torch)
    print("batched lanes", lanes, [(s["type"], tuple(s["A"].shape)) for s in specs], flush=True)
    res, infos = q.batched(specs, lanes=lanes, return_info=True)
    torch.cuda.synchronize()
    for sp, r, ex, inf in zip(specs, res, exact, infos):
        alone = _standalone(q, sp)
        assert _same(r, alone), (sp["type"], tuple(sp["A"].shape))
        vals = (r[0] if sp["type"] == "eig" else r[1]).cpu().numpy()
        e = ex[:len(vals)]
        assert np.max(np.abs(vals - e) / np.abs(e)) <= 1e-12, (sp["type"], tuple(sp["A"].shape))
        assert inf["status"] == 0


def test_batched_reports_failing_instance_and_finishes_the_rest():
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, _ = _specs(torch)
    bad = specs[1]["A"].clone()
    bad[3, 5] = float("nan")
    bad[5, 3] = float("nan")
    specs[1] = dict(type="eig", A=bad, fraction=0.2)
    print("batched with a NaN instance", flush=True)
    count = len(specs)
    probs = (q.Problem * count)()
    keep, outs = [], []
    for i, sp in enumerate(specs):
        p, kp, out = q._problem(torch, sp)
        probs[i] = p
        keep += kp
        outs.append(out)
    o = q.default_opts()
    nbytes = q.lib().qdwhp_batched_workspace(count, probs, ctypes.byref(o))
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    infos = (q.Info * count)()
    stat = (ctypes.c_int * count)()
    st = q.lib().qdwhp_batched(count, probs, ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.byref(o), 3,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), infos, stat)
    torch.cuda.synchronize()
    assert st == 1 and stat[1] == 1
    for i in [0, 2, 3, 4, 5, 6]:
        assert stat[i] == 0
        assert _same(q._result(outs[i]), _standalone(q, specs[i])), i


def test_server_alone_equals_mix_bitwise():
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = _specs(torch)
    print("server alone vs mix", flush=True)
    with q.Server(arena_bytes=2 << 30, lanes=4) as srv:
        t = srv.submit(specs[3])
        alone, info, lat, qms = srv.poll(t)
        assert lat >= 0 and qms >= 0
        tickets = [srv.submit(sp) for sp in specs]      # the same problem again, in a mix
        got = [srv.poll(tk) for tk in tickets]
    assert _same(got[3][0], alone)
    for sp, g in zip(specs, got):
        assert _same(g[0], _standalone(q, sp)), (sp["type"], tuple(sp["A"].shape))
    # and each served result is right: values against the planted spectra,
    # residuals and orthogonality of every returned vector
    _check_planted(specs, exact, [g[0] for g in got])


def _check_planted(specs, exact, results):
    import oracle
    for sp, ex, r in zip(specs, exact, results):
        A = sp["A"].cpu().numpy()
        if sp["type"] == "eig":
            w, V = (x.cpu().numpy() for x in r)
            e = ex[:len(w)]
            met = oracle.eig_metrics(A, w, V, e)
            orth = met["orth"]
        else:
            U, S, V = (x.cpu().numpy() for x in r)
            e = ex[:len(S)]
            met = oracle.svd_metrics(A, U, S, V, e)
            orth = max(met["orth_u"], met["orth_v"])
        tag = (sp["type"], tuple(sp["A"].shape))
        assert met["value_rel_max"] <= 1e-12, (tag, met)
        assert met["residual"] <= 1e-13, (tag, met)
        assert orth <= 1e-12, (tag, met)


def test_server_admission_by_footprint():
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, _ = _specs(torch)
    o = q.default_opts()
    p, keep, _ = q._problem(torch, specs[0])
    fp = q.lib().qdwhp_problem_workspace(ctypes.byref(p), ctypes.byref(o))
    print("server footprint", fp, flush=True)
    # room for one request at a time: the second waits for the first
    with q.Server(arena_bytes=int(fp * 1.5), lanes=4) as srv:
        t1 = srv.submit(specs[0])
        t2 = srv.submit(specs[0])
        from synthetic import eig_uniform
        Abig, _ = eig_uniform(600, 19, device=torch.device("cuda"))
        big = srv.submit(dict(type="eig", A=Abig, fraction=0.1))   # larger than the arena: fails at once
        r2 = srv.poll(t2)
        r1 = srv.poll(t1)
        with pytest.raises(q.QdwhpError) as e:
            srv.poll(big)
        assert e.value.status == 4
    assert _same(r1[0], r2[0])
    # FIFO: the second request queued until the first released its memory
    assert r2[3] > 0.0 and r2[2] > r1[2]


def test_server_poll_nonblocking():
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, _ = _specs(torch)
    print("server nonblocking poll", flush=True)
    with q.Server(arena_bytes=1 << 30, lanes=2) as srv:
        t = srv.submit(specs[2])
        r = None
        import time
        t0 = time.time()
        while r is None and time.time() - t0 < 60:
            r = srv.poll(t, wait=False)
            time.sleep(0.002)
        assert r is not None
