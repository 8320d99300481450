"""Complex Hermitian QDWHpartial-EIG on the GPU (qdwhp_heig, through the C
ABI) against the oracle's complex-arithmetic solve and the planted spectra.
Each case prints its name before the GPU call."""
import numpy as np
import pytest

from oracle.hermitian import heig_partial, heig_metrics
from synthetic import heig_uniform, heig_clustered, haar_complex, planted_herm, rng

pytestmark = pytest.mark.gpu

TOL_LIB = 0.05


def _gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_2104_14186_amd as q
    return torch, q


def _isolated(w, gap):
    d = np.abs(np.diff(w))
    left = np.concatenate([[np.inf], d])
    right = np.concatenate([d, [np.inf]])
    return np.minimum(left, right) > gap


@pytest.mark.parametrize("n,f,which,spec,seed", [(300, 0.1, "largest", "uniform", 71),
                                                 (400, 0.05, "largest", "clustered", 72),
                                                 (350, 0.2, "smallest", "uniform", 73),
                                                 (1100, 0.1, "largest", "clustered", 74),
                                                 (1, 1.0, "largest", "uniform", 75)])
def test_heig_vs_oracle(n, f, which, spec, seed):
    torch, q = _gpu()
    A, lam = (heig_uniform if spec == "uniform" else heig_clustered)(n, seed)
    print(f"heig n={n} f={f} which={which} {spec}", flush=True)
    w, V, info = q.eig_hermitian(torch.from_numpy(A).cuda(), f, which=which,
                                 opts=q.default_opts(tol=TOL_LIB), return_info=True)
    w, V = w.cpu().numpy(), V.cpu().numpy()
    k = len(w)
    exact = (np.sort(lam)[::-1] if which == "largest" else np.sort(lam))[:k]
    met = heig_metrics(A, w, V, exact)
    print(f"  k={k} ell(embedding)={info['ell']} {met}", flush=True)
    assert info["k"] == k
    assert met["value_rel_max"] < 1e-12
    assert met["residual"] < 1e-13, met
    assert met["orth"] < 1e-12, met
    if n > 1:
        o = heig_partial(A, fraction=f, which=which, tol=TOL_LIB)
        assert o["k"] == k
        assert np.max(np.abs(w - o["w"]) / np.abs(o["w"])) < 1e-12
        # isolated eigenvalues: the phase-normalised vectors agree
        sel = _isolated(o["w"], 1e-6 * np.abs(lam).max())
        if sel.any():
            assert np.max(np.abs(V[:, sel] - o["V"][:, sel])) < 1e-8


def test_heig_repeated_eigenvalues():
    """Complex eigenvalues of multiplicity 3 among the wanted ones (clusters
    of 6 real Ritz values): the Gram-Schmidt of the cluster keeps 3."""
    torch, q = _gpu()
    n = 240
    g = rng(76)
    lam = g.uniform(-1.0, 0.6, size=n)
    lam[:3] = 0.9
    lam[3:6] = 0.8
    lam[6:8] = 0.75
    A = planted_herm(haar_complex(g, n), lam)
    print("heig repeated eigenvalues", flush=True)
    w, V = q.eig_hermitian(torch.from_numpy(A).cuda(), 0.05, opts=q.default_opts(tol=TOL_LIB))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    k = len(w)
    exact = np.sort(lam)[::-1][:k]
    met = heig_metrics(A, w, V, exact)
    print(f"  k={k} {met}", flush=True)
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13 and met["orth"] < 1e-12
