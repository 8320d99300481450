"""QDWHpartial-EIG for complex Hermitian matrices (Sec. 4 treats real
symmetric matrices and notes that the nonreal Hermitian case carries over
with conjugate transposes).  Test infrastructure only: nothing in the
library imports it.

The steps are those of Algorithm 1 (``partial.eig_partial``) in complex
arithmetic: the estimator's Lanczos processes run on the Hermitian operator
(real Gaussian start vectors from the same Philox streams, inner products
with conjugation; the tridiagonal matrices are real), the threshold, shift
and DWH schedule are the real ones, the QR-based step factors [sqrt(c) X; I]
and forms Q1 Q2^H, the Cholesky-based step uses Z = I + c X^H X = W^H W, the
iterate is made Hermitian after every step, the projector (X + I)/2 is
factored by complex Householder QR (LAPACK through numpy), and the
Rayleigh-Ritz matrix Q2^H A Q2 is solved by LAPACK's Hermitian eigensolver.

Reading (the paper fixes no phase): every returned eigenvector is scaled by
a unit complex number that makes its largest-magnitude entry real and
positive (lowest index on ties), the complex form of the real sign rule.
"""
import numpy as np
import scipy.linalg as sla

from .dwh import eig_schedule
from .estimator import lanczos_steps, choose_tau
from .partial import wanted_count, NoSubspace, TOL, S_EIG
from .philox import gaussian


def lanczos_slq_h(op, n, seed, nv=8, m=None):
    """The estimator's Lanczos quadrature (as estimator.lanczos_slq) for a
    Hermitian operator: complex basis, conjugated inner products."""
    m = lanczos_steps(n) if m is None else m
    alpha = np.zeros((nv, m))
    beta = np.zeros((nv, m))
    for i in range(nv):
        Q = np.zeros((n, m), dtype=np.complex128)
        g = gaussian(seed, i, n).astype(np.complex128)
        Q[:, 0] = g / np.linalg.norm(g)
        amax = 0.0
        for j in range(m):
            w = op(Q[:, j])
            a = float(np.real(np.vdot(Q[:, j], w)))
            w = w - a * Q[:, j]
            if j > 0:
                w = w - beta[i, j - 1] * Q[:, j - 1]
            for _ in range(2):
                w = w - Q[:, :j + 1] @ (Q[:, :j + 1].conj().T @ w)
            bj = float(np.linalg.norm(w))
            alpha[i, j] = a
            amax = max(amax, abs(a) + (beta[i, j - 1] if j > 0 else 0.0))
            if j == m - 1:
                beta[i, j] = bj
                break
            if bj <= 1e-10 * amax:
                g = gaussian(seed, nv + i * m + j, n).astype(np.complex128)
                for _ in range(2):
                    g = g - Q[:, :j + 1] @ (Q[:, :j + 1].conj().T @ g)
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
    return dict(alpha=alpha, beta=beta, nodes=nodes, weights=weights, resid=resid, nv=nv, m=m, n=n,
                lmax=float(np.max(nodes + resid)), lmin=float(np.min(nodes - resid)))


def qr_step_h(X, a, b, c):
    """Eq. (2) with conjugate transposes: [sqrt(c) X; I] = [Q1; Q2] R,
    X+ = (b/c) X + (a - b/c)/sqrt(c) Q1 Q2^H."""
    m, n = X.shape
    Q, _ = np.linalg.qr(np.vstack([np.sqrt(c) * X, np.eye(n)]), mode="reduced")
    return (b / c) * X + (a - b / c) / np.sqrt(c) * (Q[:m] @ Q[m:].conj().T)


def chol_step_h(X, a, b, c):
    """Eq. (3) with conjugate transposes: Z = I + c X^H X = W^H W,
    X+ = (b/c) X + (a - b/c) (X W^{-1}) W^{-H} (two triangular solves)."""
    n = X.shape[1]
    W = sla.cholesky(np.eye(n) + c * (X.conj().T @ X), lower=False)
    Y1h = sla.solve_triangular(W, X.conj().T, trans="C", lower=False)    # W^{-H} X^H = (X W^{-1})^H
    Yh = sla.solve_triangular(W, Y1h, trans="N", lower=False)           # W^{-1} (X W^{-1})^H
    return (b / c) * X + (a - b / c) * Yh.conj().T


def phase_normalize(V):
    """Scale each column so that its largest-magnitude entry is real positive."""
    idx = np.argmax(np.abs(V), axis=0)
    piv = V[idx, np.arange(V.shape[1])]
    return V * (np.abs(piv) / piv)[None, :]


def heig_partial(A, fraction=None, k=None, which="largest", seed=0, s=S_EIG, iters=3, tol=TOL,
                 kappa_max=100.0, tau_policy="cost", nv=None, m=None):
    """Wanted eigenpairs of the complex Hermitian A (k mode): the k largest
    ('largest') or smallest ('smallest').  Returns dict with w (most wanted
    first), V (n x k complex, phase-normalised) and the intermediates."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Aw = -A if which == "smallest" else A
    kw = {} if nv is None else {"nv": nv}
    if m is not None:
        kw["m"] = m
    est = lanczos_slq_h(lambda v: Aw @ v, n, seed, **kw)
    if k is None:
        k = wanted_count(n, fraction)
    I = np.eye(n)
    for boost in (1, 2):
        tau, mu, rho = choose_tau(est, k, boost, tau_policy, s, iters, kappa_max, tol)
        sched = eig_schedule(s, rho, iters, kappa_max)
        X = ((1.0 - s) / mu) * (tau * I - Aw) - s * I
        for st in sched:
            step = qr_step_h if st["kind"] == "qr" else chol_step_h
            X = step(X, st["a"], st["b"], st["c"])
            X = 0.5 * (X + X.conj().T)
        B = 0.5 * (X + I)
        Q, R = np.linalg.qr(B, mode="complete")
        d = np.abs(np.diag(R))
        small = np.nonzero(d < tol)[0]
        if len(small) == 0:
            continue
        ind = int(small[0]) + 1
        ell = n - ind + 1
        Q2 = Q[:, ind - 1:]
        H = Q2.conj().T @ (Aw @ Q2)
        H = 0.5 * (H + H.conj().T)
        theta, W = np.linalg.eigh(H)
        theta, W = theta[::-1].copy(), W[:, ::-1].copy()
        n_above = int(np.sum(theta >= tau))
        if n_above >= k or ell >= n:
            break
    else:
        raise NoSubspace("fewer than k Ritz values above the threshold")
    if ell < k:
        raise NoSubspace("subspace smaller than k")
    V = phase_normalize(Q2 @ W[:, :k])
    lam = theta[:k].copy()
    if which == "smallest":
        lam = -lam
    return dict(w=lam, V=V, k=k, tau=tau, mu=mu, rho=rho, sched=sched, ind=ind, ell=ell, diagR=np.diag(R),
                theta=theta, est=est, X=X)


def heig_metrics(A, w, V, exact=None):
    """Sec. 7.3's metrics for Hermitian A: max_i ||A v_i - w_i v_i|| / ||A||_2,
    ||I - V^H V||_F, and the max relative value error against ``exact``."""
    A = np.asarray(A)
    nrm = np.linalg.norm(A, 2)
    res = float(np.max(np.linalg.norm(A @ V - V * w[None, :], axis=0)) / nrm) if V.shape[1] else 0.0
    orth = float(np.linalg.norm(np.eye(V.shape[1]) - V.conj().T @ V))
    out = dict(residual=res, orth=orth)
    if exact is not None:
        out["value_rel_max"] = float(np.max(np.abs(w - exact) / np.abs(exact)))
    return out
