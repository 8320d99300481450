"""Spectrum bounds and the wanted threshold from a few Lanczos steps.

Algorithm 1 starts with a few Lanczos steps to bound the spectrum (Sec. 4.1),
and Algorithm 2 with a norm estimate alpha of ||A||_2 (Sec. 4.2).  The paper's
interface is threshold-based (negative eigenvalues; singular values above
s ||A||_2).  To serve a *fraction* of the spectrum, the same Lanczos runs are
read as a stochastic Lanczos quadrature of the spectral counting function, and
the threshold is placed so that an estimated k_t >= k eigenvalues lie above it.
The paper is silent on this mapping; the reading below is used by both the
oracle and the HIP path, and the solver checks the result a posteriori (the
number of Rayleigh-Ritz values above the threshold must be at least k, which by
interlacing certifies that the top-k values are among those captured).

Lanczos definition (both sides):
  * nv independent runs of m steps; run i starts from the Philox Gaussian
    stream i, normalised;
  * three-term recurrence with full re-orthogonalisation (classical
    Gram-Schmidt applied twice);
  * if beta_j <= 1e-10 * max_{i<=j}(|alpha_i| + beta_{i-1}) the run restarts
    from the Philox stream nv + i*m + j, orthogonalised twice against the run's
    basis, and beta_j is set to 0;
  * T = tridiag(alpha, beta_1..beta_{m-1}); Ritz values theta, quadrature
    weights (first eigenvector component)^2, residual bounds |beta_m y_m|.
"""
import math
import numpy as np
import scipy.linalg as sla

from .philox import gaussian
from .dwh import compose, eig_schedule

NV_DEFAULT = 8
M_DEFAULT = 64


def lanczos_steps(n, m_default=M_DEFAULT):
    return max(1, min(m_default, n - 1))


def lanczos_slq(op, n, seed, nv=NV_DEFAULT, m=None):
    """Run ``nv`` Lanczos processes of ``m`` steps on the symmetric operator ``op``.

    Returns dict with per-run alpha (nv, m), beta (nv, m) (beta[:, m-1] is the
    final residual norm) and the pooled Ritz nodes, weights and residual bounds.
    """
    m = lanczos_steps(n) if m is None else m
    alpha = np.zeros((nv, m))
    beta = np.zeros((nv, m))
    for i in range(nv):
        Q = np.zeros((n, m))
        g = gaussian(seed, i, n)
        Q[:, 0] = g / np.linalg.norm(g)
        amax = 0.0
        for j in range(m):
            w = op(Q[:, j])
            a = float(Q[:, j] @ w)
            w = w - a * Q[:, j]
            if j > 0:
                w = w - beta[i, j - 1] * Q[:, j - 1]
            for _ in range(2):
                w = w - Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
            bj = float(np.linalg.norm(w))
            alpha[i, j] = a
            amax = max(amax, abs(a) + (beta[i, j - 1] if j > 0 else 0.0))
            if j == m - 1:
                beta[i, j] = bj
                break
            if bj <= 1e-10 * amax:
                g = gaussian(seed, nv + i * m + j, n)
                for _ in range(2):
                    g = g - Q[:, :j + 1] @ (Q[:, :j + 1].T @ g)
                Q[:, j + 1] = g / np.linalg.norm(g)
                beta[i, j] = 0.0
            else:
                Q[:, j + 1] = w / bj
                beta[i, j] = bj
    nodes, weights, resid = [], [], []
    for i in range(nv):
        if m == 1:
            th, Y = alpha[i, :1].copy(), np.ones((1, 1))
        else:
            th, Y = sla.eigh_tridiagonal(alpha[i], beta[i, :m - 1])
        nodes.append(th)
        weights.append(Y[0, :] ** 2)
        resid.append(np.abs(beta[i, m - 1] * Y[m - 1, :]))
    nodes = np.concatenate(nodes)
    weights = np.concatenate(weights)
    resid = np.concatenate(resid)
    return dict(alpha=alpha, beta=beta, nodes=nodes, weights=weights, resid=resid,
                nv=nv, m=m, n=n,
                lmax=float(np.max(nodes + resid)), lmin=float(np.min(nodes - resid)))


def count_above(est, t):
    """Quadrature estimate of #{eigenvalues >= t}."""
    return est["n"] / est["nv"] * float(np.sum(est["weights"][est["nodes"] >= t]))


def target_count(n, k, boost=1):
    """k_t = k + max(16, ceil(k/10)), multiplied by ``boost`` on a retry, capped at n."""
    return min(n, boost * (k + max(16, int(math.ceil(0.1 * k)))))


def _cut_below(est, kt, nonneg=False):
    """Threshold below the node at which the estimated count first reaches kt.

    Nodes are pooled over the runs and sorted downwards; the cut is placed
    halfway between that node and the next node that is distinct from it
    (more than 1e-6 of the estimated spectral spread below), so a cluster that
    several runs resolve as one node is kept whole.  Returns None if the count
    never reaches kt (everything wanted).

    nonneg (nodes of A^T A, which span many decades when A is ill
    conditioned): a node is distinct when it lies more than 1e-6 of the
    node's own value below, and when no node is, the cut is halfway down to
    the spectrum's lower end 0.
    """
    order = np.argsort(-est["nodes"], kind="stable")
    th = est["nodes"][order]
    cum = est["n"] / est["nv"] * np.cumsum(est["weights"][order])
    hit = np.nonzero(cum >= kt - 1e-9)[0]
    if len(hit) == 0 or kt >= est["n"]:
        return None
    j = int(hit[0])
    spread = max(est["lmax"] - est["lmin"], abs(est["lmax"]), abs(est["lmin"]), 1e-300)
    gap = 1e-6 * abs(th[j]) if nonneg else 1e-6 * spread
    below = th[j + 1:][th[j + 1:] < th[j] - gap]
    if len(below) == 0:
        return 0.5 * th[j] if (nonneg and th[j] > 0.0) else None
    nxt = max(float(below[0]), 0.0) if nonneg else float(below[0])
    return 0.5 * (th[j] + nxt)


def _band_edge(sched, s, tol):
    """Scaled value y in (-s, 0) where the composite map of the EIG schedule
    reaches 2 tol - 1, i.e. (r(y) + 1)/2 = tol: scaled values above it are
    the band the projector keeps beyond the wanted part (Sec. 4.1)."""
    ws = [(st["a"], st["b"], st["c"]) for st in sched]
    target = 2.0 * tol - 1.0
    lo, hi = -s, 0.0
    if not compose(lo, ws) < target:
        return lo
    for _ in range(200):
        if hi - lo <= 1e-17:
            break
        mid = 0.5 * (lo + hi)
        if compose(mid, ws) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def predicted_flops(sched, n, ell):
    """Table 1 accounting of one EIG solve with the given step kinds and
    subspace size: (8 + 2/3) n^3 per QR-based and (4 + 1/3) n^3 per
    Cholesky-based step, the Householder QR of the projector's first
    j = n - ell columns (2 n j^2 - 2/3 j^3), A Q2 plus forming Q2 (6 n^2 ell)
    and the ell x ell eigenproblem (9 ell^3)."""
    n = float(n)
    ell = float(ell)
    f = sum((26.0 / 3.0 if st["kind"] == "qr" else 13.0 / 3.0) * n ** 3 for st in sched)
    j = max(0.0, n - ell)
    return f + 2.0 * n * j * j - 2.0 / 3.0 * j ** 3 + 6.0 * n * n * ell + 9.0 * ell ** 3


def _scale(est, tau):
    spread = max(est["lmax"] - est["lmin"], abs(est["lmax"]), abs(est["lmin"]), 1e-300)
    mu = max(est["lmax"] - tau, 1e-3 * spread)
    rho = max(0.0, (tau - est["lmin"]) / mu)
    return mu, rho


def choose_tau(est, k, boost=1, policy="cost", s=0.2, iters=3, kappa_max=100.0, tol=0.01):
    """EIG threshold tau and scaling for the wanted top-k (Algorithm 1 setup).

    Returns (tau, mu, rho): |mu| = lambda_max_hat - tau scales the wanted part
    onto [-1, 0] (Sec. 4.1 scales by a Lanczos bound), rho = (tau - lambda_min_hat)/|mu|
    bounds the largest unwanted scaled value.

    policy 'plain': tau is the cut below the target count (``_cut_below``).
    policy 'cost' (reading; the paper leaves the threshold to the user and
    notes the trade-off between QR- and Cholesky-based steps): every cut at
    or below the plain one that lies in a gap between distinct quadrature
    nodes is a candidate; for each, the step kinds follow from rho
    (``eig_schedule``), the subspace size ell is predicted as the quadrature
    count above the band edge, and ``predicted_flops`` scores it; the
    cheapest wins, ties going to the higher cut.
    """
    n = est["n"]
    kt = target_count(n, k, boost)
    if policy == "plain":
        cut = _cut_below(est, kt)
        tau = est["lmin"] if cut is None else cut
        mu, rho = _scale(est, tau)
        return tau, mu, rho
    order = np.argsort(-est["nodes"], kind="stable")
    th = est["nodes"][order]
    cum = n / est["nv"] * np.cumsum(est["weights"][order])
    hit = np.nonzero(cum >= kt - 1e-9)[0]
    if len(hit) == 0 or kt >= n:
        mu, rho = _scale(est, est["lmin"])
        return est["lmin"], mu, rho
    spread = max(est["lmax"] - est["lmin"], abs(est["lmax"]), abs(est["lmin"]), 1e-300)
    gap = 1e-6 * spread
    j = int(hit[0])
    best = None
    while True:
        below = np.nonzero(th[j + 1:] < th[j] - gap)[0]
        if len(below) == 0:
            break
        nx = j + 1 + int(below[0])
        tau = 0.5 * (th[j] + th[nx])
        mu, rho = _scale(est, tau)
        sched = eig_schedule(s, rho, iters, kappa_max)
        edge = tau - mu * (_band_edge(sched, s, tol) + s) / (1.0 - s)
        ell = min(float(n), count_above(est, edge))
        cost = predicted_flops(sched, n, ell)
        if best is None or cost < best[0] * (1.0 - 1e-12):
            best = (cost, tau, mu, rho)
        j = nx
    if best is None:
        mu, rho = _scale(est, est["lmin"])
        return est["lmin"], mu, rho
    return best[1], best[2], best[3]


def choose_svd_threshold(est, k, boost=1):
    """SVD norm estimate alpha and relative threshold s (Algorithm 2 setup).

    ``est`` comes from Lanczos on A^T A, so nodes are squared singular values.
    alpha = sqrt(lambda_max_hat(A^T A)); s = sqrt(t)/alpha with t the cut for
    the wanted count, clamped to [1e-15, 1].
    """
    n = est["n"]
    alpha = math.sqrt(max(est["lmax"], 0.0))
    if alpha == 0.0:
        alpha = 1e-300
    kt = target_count(n, k, boost)
    cut = _cut_below(est, kt, nonneg=True)
    t = 0.0 if cut is None else max(cut, 0.0)
    s = min(1.0, max(1e-15, math.sqrt(t) / alpha))
    return alpha, s
