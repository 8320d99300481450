"""Seeded generators for the planted-spectrum workloads.

Every matrix is A = Q diag(lambda) Q^T (symmetric) or A = U diag(sigma) V^T
(general) with Haar-distributed orthogonal factors, so the exact eigen/singular
values are known.  The paper builds its test matrices the same way (Sec. 7.2:
A = Q1 D Q2^T from QR factors of random matrices, Q1 = Q2 for the symmetric
case); the spectra used here are the planted ones of the benchmark workloads.

Draw order is fixed: orthogonal factors first, then the spectrum.  The
generator is numpy's PCG64 so the same seed yields the same Gaussian draws on
any host.  When ``device`` is a torch CUDA/HIP device, the Gaussian draws are
still made by numpy and only the QR and the final product run there (this is
input construction, not part of the solver), which keeps 16K-sized inputs
cheap to build.
"""
import numpy as np

CONFIG_SEEDS = {"eig512": 1000, "svd4096": 1001, "eig16384": 1002,
                "svd16384x8192": 1003, "trace": 4000, "pool": 41000}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _sign_fix_np(Q, R):
    d = np.sign(np.diag(R)).copy()
    d[d == 0] = 1.0
    return Q * d[None, :]


def haar(g, m, n=None, device=None):
    """Haar-distributed m x n matrix with orthonormal columns (n <= m).

    QR of a Gaussian matrix with the signs of diag(R) moved into Q.
    """
    n = m if n is None else n
    G = g.standard_normal((m, n))
    if device is None:
        Q, R = np.linalg.qr(G)
        return _sign_fix_np(Q, R)
    import torch
    Gt = torch.from_numpy(G).to(device)
    Q, R = torch.linalg.qr(Gt)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def planted_sym(Q, lam):
    """A = Q diag(lam) Q^T, symmetrised exactly."""
    if isinstance(Q, np.ndarray):
        A = (Q * lam[None, :]) @ Q.T
        return 0.5 * (A + A.T)
    import torch
    lt = torch.as_tensor(lam, dtype=Q.dtype, device=Q.device)
    A = (Q * lt[None, :]) @ Q.T.contiguous()
    return 0.5 * (A + A.T)


def planted_general(U, sigma, V):
    """A = U diag(sigma) V^T."""
    if isinstance(U, np.ndarray):
        return (U * sigma[None, :]) @ V.T
    import torch
    st = torch.as_tensor(sigma, dtype=U.dtype, device=U.device)
    return (U * st[None, :]) @ V.T.contiguous()


def eig_uniform(n, seed, lo=-1.0, hi=1.0, device=None):
    """Symmetric n x n, eigenvalues i.i.d. uniform on [lo, hi]."""
    g = rng(seed)
    Q = haar(g, n, device=device)
    lam = g.uniform(lo, hi, size=n)
    return planted_sym(Q, lam), lam


def eig_clustered(n, seed, bulk_frac=0.9, bulk=(-1.0, 0.5), top=(0.5, 1.0),
                  nclusters=8, width=1e-8, device=None):
    """Symmetric n x n: a uniform bulk plus tight clusters in the top interval.

    ``bulk_frac`` of the eigenvalues are uniform on ``bulk``; the rest are split
    into ``nclusters`` clusters of width ``width`` whose centres are evenly
    spaced in ``top`` (centre j at lo + (j + 1/2) (hi - lo) / nclusters).
    Cluster sizes differ by at most one (larger clusters first).
    """
    g = rng(seed)
    Q = haar(g, n, device=device)
    nb = int(round(bulk_frac * n))
    nc = n - nb
    lam_b = g.uniform(bulk[0], bulk[1], size=nb)
    sizes = [nc // nclusters + (1 if j < nc % nclusters else 0) for j in range(nclusters)]
    parts = [lam_b]
    for j, sz in enumerate(sizes):
        c = top[0] + (j + 0.5) * (top[1] - top[0]) / nclusters
        parts.append(c + g.uniform(-0.5 * width, 0.5 * width, size=sz))
    lam = np.concatenate(parts)
    return planted_sym(Q, lam), lam


def haar_complex(g, n, device=None):
    """Haar-distributed n x n unitary: QR of a complex Gaussian matrix with
    the phases of diag(R) moved into Q (on ``device`` with torch when given)."""
    G = (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))) / np.sqrt(2.0)
    if device is None:
        Q, R = np.linalg.qr(G)
        d = np.diag(R)
        ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
        return Q * ph[None, :]
    import torch
    Q, R = torch.linalg.qr(torch.from_numpy(G).to(device))
    d = torch.diagonal(R)
    ph = torch.where(d.abs() > 0, d / d.abs(), torch.ones_like(d))
    return Q * ph[None, :]


def planted_herm(Q, lam):
    """A = Q diag(lam) Q^H, made Hermitian exactly."""
    if isinstance(Q, np.ndarray):
        A = (Q * lam[None, :]) @ Q.conj().T
        return 0.5 * (A + A.conj().T)
    import torch
    lt = torch.as_tensor(lam, dtype=Q.dtype, device=Q.device)
    A = (Q * lt[None, :]) @ Q.conj().t().contiguous()
    return 0.5 * (A + A.conj().t())


def heig_uniform(n, seed, lo=-1.0, hi=1.0, device=None):
    """Complex Hermitian n x n, eigenvalues i.i.d. uniform on [lo, hi]."""
    g = rng(seed)
    Q = haar_complex(g, n, device)
    lam = g.uniform(lo, hi, size=n)
    return planted_herm(Q, lam), lam


def heig_clustered(n, seed, bulk_frac=0.9, bulk=(-1.0, 0.5), top=(0.5, 1.0), nclusters=8, width=1e-8,
                   device=None):
    """Complex Hermitian counterpart of eig_clustered (same spectrum recipe)."""
    g = rng(seed)
    Q = haar_complex(g, n, device)
    nb = int(round(bulk_frac * n))
    nc = n - nb
    lam_b = g.uniform(bulk[0], bulk[1], size=nb)
    sizes = [nc // nclusters + (1 if j < nc % nclusters else 0) for j in range(nclusters)]
    parts = [lam_b]
    for j, sz in enumerate(sizes):
        c = top[0] + (j + 0.5) * (top[1] - top[0]) / nclusters
        parts.append(c + g.uniform(-0.5 * width, 0.5 * width, size=sz))
    lam = np.concatenate(parts)
    return planted_herm(Q, lam), lam


def svd_geometric(m, n, seed, kappa=1e16, device=None):
    """m x n (m >= n), sigma_i = kappa^{-(i-1)/(n-1)} (geometric, 1 .. 1/kappa)."""
    g = rng(seed)
    U = haar(g, m, n, device=device)
    V = haar(g, n, device=device)
    i = np.arange(n, dtype=np.float64)
    sigma = kappa ** (-(i / max(n - 1, 1)))
    return planted_general(U, sigma, V), sigma


def svd_loguniform(m, n, seed, lo_exp=-6.0, hi_exp=0.0, device=None):
    """m x n (m >= n), sigma = sort_desc(10^{U[lo_exp, hi_exp]})."""
    g = rng(seed)
    U = haar(g, m, n, device=device)
    V = haar(g, n, device=device)
    sigma = np.sort(10.0 ** g.uniform(lo_exp, hi_exp, size=n))[::-1].copy()
    return planted_general(U, sigma, V), sigma


def request_trace(nreq, rate, seed, sizes=(256, 512, 1024, 2048, 4096),
                  eig_frac=0.6, frac_range=(0.01, 0.20), log_kappa_max=12.0):
    """Mixed stream of partial-spectrum requests with Poisson arrivals.

    Returns a list of dicts: kind ('eig'|'svd'), n, fraction, k, arrival (s),
    matrix seed and, for SVD, kappa.  Matrices are built lazily by the caller
    from (kind, n, seed) so a trace stays small.
    """
    g = rng(seed)
    t = 0.0
    out = []
    for r in range(nreq):
        t += g.exponential(1.0 / rate)
        kind = "eig" if g.uniform() < eig_frac else "svd"
        n = int(sizes[g.integers(len(sizes))])
        f = float(g.uniform(*frac_range))
        k = max(1, int(np.floor(f * n + 0.5)))
        kappa = float(10.0 ** g.uniform(0.0, log_kappa_max))
        out.append(dict(kind=kind, n=n, fraction=f, k=k, arrival=t,
                        seed=CONFIG_SEEDS["pool"] + r, kappa=kappa))
    return out
