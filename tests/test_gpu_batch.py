"""Ragged batches, the persistent grouped GEMM and the request server.

Batches and the server run the DWH iterations of instances of one shape as
grouped launches (grouped Gram, lockstep Cholesky-inversion with batched
leaves, grouped triangular products).  Each grouped launch performs every
member's operations exactly as its standalone call would, so batched and
served results equal standalone calls bitwise, alone and in any batch or mix.
Values are checked against the planted spectra, and every returned vector's
residual and orthogonality.  Each case prints its shapes before GPU work."""
import contextlib
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


def _specs_same_shape(torch):
    """Groups of equal shapes (so the iterations really run grouped): three
    EIG of n = 256, two of n = 384 (smallest), three SVD of 300 x 200."""
    from synthetic import eig_uniform, svd_geometric
    dev = torch.device("cuda")
    specs, exact = [], []
    for seed, f in [(61, 0.1), (62, 0.2), (63, 0.05)]:
        A, lam = eig_uniform(256, seed, device=dev)
        specs.append(dict(type="eig", A=A, fraction=f))
        exact.append(np.sort(lam)[::-1])
    for seed in (64, 65):
        A, lam = eig_uniform(384, seed, device=dev)
        specs.append(dict(type="eig", A=A, fraction=0.1, which="smallest"))
        exact.append(np.sort(lam))
    for seed, kappa in [(66, 1e3), (67, 1e8), (68, 1e12)]:
        A, sg = svd_geometric(300, 200, seed, kappa=kappa, device=dev)
        specs.append(dict(type="svd", A=A, k=12))
        exact.append(np.asarray(sg))
    return specs, exact


def _standalone(q, sp):
    if sp["type"] == "eig":
        return q.eig(sp["A"], fraction=sp["fraction"], which=sp.get("which", "largest"))
    return q.svd(sp["A"], sp["k"])


def _same(a, b):
    return all(bool((x == y).all()) for x, y in zip(a, b))


@contextlib.contextmanager
def _tuned(q, **keys):
    old = {k: q.tune_get(k.replace("_", "."), -12345) for k in keys}
    try:
        for k, v in keys.items():
            q.tune_set(k.replace("_", "."), v)
        yield
    finally:
        for k, v in old.items():
            if v == -12345:
                q.tune_set(k.replace("_", "."), 1)
            else:
                q.tune_set(k.replace("_", "."), v)


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


@pytest.mark.parametrize("lanes,same", [(1, False), (4, False), (2, True), (4, True)])
def test_batched_equals_standalone_bitwise(lanes, same):
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = (_specs_same_shape if same else _specs)(torch)
    print("batched lanes", lanes, [(s["type"], tuple(s["A"].shape)) for s in specs], flush=True)
    res, infos = q.batched(specs, lanes=lanes, return_info=True)
    torch.cuda.synchronize()
    _check_planted(specs, exact, res)
    for sp, r, inf in zip(specs, res, infos):
        assert inf["status"] == 0
        assert _same(r, _standalone(q, sp)), (sp["type"], tuple(sp["A"].shape))


def test_batched_result_does_not_depend_on_the_batch():
    """The same instance in two different batches (and alone in a batch):
    bitwise the same result."""
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = _specs_same_shape(torch)
    print("batch composition", flush=True)
    full = q.batched(specs, lanes=3)
    part = q.batched([specs[5], specs[0], specs[2]], lanes=2)
    one = q.batched([specs[2]], lanes=1)
    torch.cuda.synchronize()
    assert _same(full[5], part[0]) and _same(full[0], part[1]) and _same(full[2], part[2])
    assert _same(full[2], one[0])


def test_batched_ungrouped_equals_standalone_bitwise():
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = _specs(torch)
    print("batched ungrouped", flush=True)
    with _tuned(q, batch_grouped=0):
        res = q.batched(specs, lanes=4)
        torch.cuda.synchronize()
        for sp, r in zip(specs, res):
            assert _same(r, _standalone(q, sp)), (sp["type"], tuple(sp["A"].shape))


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
    clean = q.batched([specs[i] for i in [0, 2, 3, 4, 5, 6]], lanes=3)
    torch.cuda.synchronize()
    for j, i in enumerate([0, 2, 3, 4, 5, 6]):
        assert stat[i] == 0
        assert _same(q._result(outs[i]), clean[j]), i


@pytest.mark.parametrize("same", [False, True])
def test_server_alone_equals_mix_bitwise(same):
    """Every request served alone (one at a time) and served in a mix with all
    the others (same-shape requests grouped): bitwise the same result, equal
    to a standalone call; each result is right (planted values, residual and
    orthogonality of every returned vector)."""
    torch = _torch()
    import paper_2104_14186_amd as q
    specs, exact = (_specs_same_shape if same else _specs)(torch)
    print("server alone vs mix", flush=True)
    with q.Server(arena_bytes=2 << 30, lanes=3) as srv:
        alone = []
        for sp in specs:
            r, info, lat, qms = srv.poll(srv.submit(sp))
            assert lat >= 0 and qms >= 0
            alone.append(r)
        tickets = [srv.submit(sp) for sp in specs]      # the same problems again, in a mix
        got = [srv.poll(tk) for tk in tickets]
    for sp, g, a in zip(specs, got, alone):
        assert _same(g[0], a), (sp["type"], tuple(sp["A"].shape))
        assert _same(g[0], _standalone(q, sp)), (sp["type"], tuple(sp["A"].shape))
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
