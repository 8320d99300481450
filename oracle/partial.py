"""QDWHpartial-EIG (Algorithm 1) and QDWHpartial-SVD (Algorithm 2), step by step.

Both functions expose every intermediate (threshold, schedule, iterates' final
X, diag(R) of the projector QR, ind, ell, Q2, the Rayleigh-Ritz matrix and
values) and accept a ``replay`` dict that fixes the estimator's outputs and the
step kinds, so an external implementation can be compared on an identical
schedule.

Readings (the paper is silent or ambiguous on these):
  * fraction -> k = floor(f n + 1/2), 1 <= k <= n; 'smallest' works on -A and
    negates the values at the end (shift/negation, Sec. 4.1);
  * the wanted part is the top-k; the threshold comes from the Lanczos
    quadrature (oracle.estimator) and is certified a posteriori;
  * EIG scaling: Btil = ((1-s)/|mu|)(tau I - A) - s I, s = 0.2, three steps
    from l_0 = s (Algorithm 1 with the shift written as (1-s)A - sI, Sec. 4.1);
  * X_k is symmetrised after every EIG step (it is symmetric in exact
    arithmetic); the Rayleigh-Ritz matrix is symmetrised too;
  * the threshold tol is applied to |R_ii| of the QR of (r+I)/2 (EIG) or
    I - r^T r (SVD), with the paper's default tol = 0.01 (Sec. 4.1 after
    Theorem 1, Algorithms 1 and 2).  Sec. 4.1 notes that a small tol costs
    accuracy and a large one costs subspace size: by Theorem 1 the
    containment error is about ||V0^T B|| / sigma_min(R11), and with
    sigma_min(R11) near 0.01 rounding in B alone can leave residuals just
    above 1e-13 (kappa = 1e16 SVD inputs); tol is a parameter of every
    entry point.  ind is 1-based, ell = n - ind + 1, no entry below tol
    means ell = 0;
  * Rayleigh-Ritz uses the original A (no rescaling), keeps the k largest
    Ritz values (EIG) / singular values (SVD);
  * the small SVD of A Q2 is QR followed by the SVD of the ell x ell R factor;
  * V is returned (not V^T); each output vector is sign-normalised so that its
    largest-magnitude entry (lowest index on ties) is positive; for the SVD the
    sign is set on V and mirrored onto U;
  * m < n: the algorithm runs on A^T and swaps U and V (Sec. 4.2).
"""
import math
import numpy as np
import scipy.linalg as sla

from .dwh import eig_schedule, svd_schedule, QR_FIRST_BELOW
from .polar import qr_step, chol_step
from .zolo import zolo_schedule, zolo_step
from .estimator import lanczos_slq, choose_tau, choose_svd_threshold
from .philox import gaussian

S_EIG = 0.2
TOL = 0.01          # Sec. 4.1 / Algorithms 1 and 2


class NoSubspace(RuntimeError):
    """Fewer than k certified values after the retry (status +2)."""


def wanted_count(n, fraction):
    return min(n, max(1, int(math.floor(fraction * n + 0.5))))


def sign_normalize(V, U=None):
    """Flip columns so the largest-|entry| of each column of V is positive."""
    idx = np.argmax(np.abs(V), axis=0)
    sg = np.where(V[idx, np.arange(V.shape[1])] < 0, -1.0, 1.0)
    V = V * sg[None, :]
    if U is not None:
        U = U * sg[None, :]
    return V, U


def omega_matrix(n, seed):
    """n x n Gaussian Omega of the randomised rank-revealing QR (Sec. 4.1),
    Philox stream 0 under key seed + 3, filled column by column.

    Reading: the entries are scaled to variance 1/n so that B Omega keeps the
    column norms of B on average and the absolute tol on |R_ii| keeps its
    meaning (with unit variance every diagonal entry grows by ~sqrt(n), the
    cut moves and the subspace loses part of the wanted space)."""
    return gaussian(seed + 3, 0, n * n).reshape((n, n), order="F") / np.sqrt(n)


def projector_subspace(B, tol=TOL, omega=None):
    """Householder QR of the projector B (no pivoting), ind and Q2 (Sec. 4.1,
    'Choosing the subspace size ell'; Algorithm 1 and Algorithm 2).  With
    ``omega`` the QR is of B Omega, which Sec. 4.1 offers to make the
    factorisation rank revealing with high probability (B Omega has the
    range of B)."""
    n = B.shape[0]
    if omega is not None:
        B = B @ omega
    Q, R = np.linalg.qr(B, mode="complete")
    d = np.abs(np.diag(R))
    small = np.nonzero(d < tol)[0]
    if len(small) == 0:
        return dict(diagR=np.diag(R).copy(), ind=n + 1, ell=0, Q2=np.zeros((n, 0)))
    ind = int(small[0]) + 1          # 1-based
    ell = n - ind + 1
    return dict(diagR=np.diag(R).copy(), ind=ind, ell=ell, Q2=Q[:, ind - 1:])


def _eig_core(Aw, tau, mu, rho, s, iters, tol, kappa_max, symmetrize, kinds=None, omega=None, zolo_r=0):
    """Steps of Algorithm 1 after the setup: iterate, project, Rayleigh-Ritz.
    zolo_r > 0: Zolotarev steps of type (2r+1, 2r) instead of DWH steps
    (oracle.zolo), from l_0 = s to convergence."""
    n = Aw.shape[0]
    if zolo_r:
        sched = zolo_schedule(s, zolo_r, kappa_max, x0=max(1.0, (1.0 - s) * rho - s))
    else:
        sched = eig_schedule(s, rho, iters, kappa_max)
        if kinds is not None:
            for st, kd in zip(sched, kinds):
                st["kind"] = kd
    # Scaled and shifted matrix (Sec. 4.1): wanted eigenvalues land in [-1, -s].
    X = ((1.0 - s) / mu) * (tau * np.eye(n) - Aw) - s * np.eye(n)
    for st in sched:
        if zolo_r:
            X = zolo_step(X, st)
        else:
            step = qr_step if st["kind"] == "qr" else chol_step
            X = step(X, st["a"], st["b"], st["c"])
        if symmetrize:
            X = 0.5 * (X + X.T)
    B = 0.5 * (X + np.eye(n))
    sub = projector_subspace(B, tol, omega)
    out = dict(tau=tau, mu=mu, rho=rho, sched=sched, X=X, B=B, **sub)
    if sub["ell"] == 0:
        out.update(theta=np.zeros(0), W=np.zeros((0, 0)), H=np.zeros((0, 0)), n_above=0)
        return out
    Q2 = sub["Q2"]
    H = Q2.T @ (Aw @ Q2)
    H = 0.5 * (H + H.T)
    theta, W = np.linalg.eigh(H)
    out.update(theta=theta[::-1].copy(), W=W[:, ::-1].copy(), H=H,
               n_above=int(np.sum(theta >= tau)))
    return out


def eig_partial(A, fraction=None, k=None, which="largest", seed=0, replay=None,
                tau=None, s=S_EIG, iters=3, tol=TOL, kappa_max=100.0, symmetrize=True,
                nv=None, m=None, tau_policy="cost", use_omega=False, zolo_r=0):
    """Wanted eigenpairs of symmetric A by QDWHpartial-EIG (Algorithm 1).

    k mode (``fraction`` or ``k``): the k largest ('largest') or smallest
    ('smallest') eigenpairs.  Threshold mode (``tau`` given, no k): every
    eigenpair beyond tau on the wanted side, the paper's native form (negative
    eigenvalues for tau = 0 and 'smallest').  Returns dict with w (most wanted
    first), V (n x k) and the intermediates.  Raises NoSubspace when the
    certificate fails after one retry (k mode).  ``tau_policy`` picks the
    k-mode threshold ('cost' or 'plain', see estimator.choose_tau);
    ``use_omega`` factors B Omega instead of B (Sec. 4.1); ``zolo_r`` > 0
    iterates Zolotarev steps of type (2 zolo_r + 1, 2 zolo_r) (oracle.zolo)
    and then takes the plain threshold cut.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Aw = -A if which == "smallest" else A
    kw = {} if nv is None else {"nv": nv}
    if m is not None:
        kw["m"] = m
    kinds = None if replay is None else replay.get("kinds")
    omega = omega_matrix(n, seed) if use_omega else None
    est = None
    if replay is None:
        est = lanczos_slq(lambda v: Aw @ v, n, seed, **kw)
    if k is None and fraction is None:
        # Threshold mode.
        if tau is None:
            raise ValueError("give fraction, k or tau")
        tw = -tau if which == "smallest" else tau
        if replay is not None:
            mu, rho = replay["mu"], replay["rho"]
        else:
            spread = max(est["lmax"] - est["lmin"], abs(est["lmax"]), abs(est["lmin"]), 1e-300)
            mu = max(est["lmax"] - tw, 1e-3 * spread)
            rho = max(0.0, (tw - est["lmin"]) / mu)
        r = _eig_core(Aw, tw, mu, rho, s, iters, tol, kappa_max, symmetrize, kinds, omega, zolo_r)
        k = r["n_above"]
    else:
        if k is None:
            k = wanted_count(n, fraction)
        for boost in (1, 2):
            if replay is not None:
                tw, mu, rho = replay["tau"], replay["mu"], replay["rho"]
            else:
                tw, mu, rho = choose_tau(est, k, boost, "plain" if zolo_r else tau_policy, s, iters,
                                         kappa_max, tol)
            r = _eig_core(Aw, tw, mu, rho, s, iters, tol, kappa_max, symmetrize, kinds, omega, zolo_r)
            if r["ell"] > 0 and (r["n_above"] >= k or r["ell"] >= n or replay is not None):
                break
        else:
            raise NoSubspace("fewer than k Ritz values above the threshold")
        if r["ell"] < k:
            raise NoSubspace("subspace smaller than k")
    V = r["Q2"] @ r["W"][:, :k] if k > 0 else np.zeros((n, 0))
    V, _ = sign_normalize(V)
    lam = r["theta"][:k].copy()
    if which == "smallest":
        lam = -lam
    r.update(w=lam, V=V, k=k, est=est)
    return r


def _svd_core(A, alpha, s, tol, kappa_max, qr_first, kinds=None, zolo_r=0):
    """Steps of Algorithm 2 after the norm estimate: iterate, project, small SVD.
    zolo_r > 0: Zolotarev steps (oracle.zolo); qr_first as for the DWH
    schedule (None: forced when s < 1e-3, Sec. 4.2)."""
    n = A.shape[1]
    if zolo_r:
        force = (float(s) < QR_FIRST_BELOW) if qr_first is None else bool(qr_first)
        sched = zolo_schedule(s, zolo_r, kappa_max, 1.0, qr_first=force)
    else:
        sched = svd_schedule(s, kappa_max, qr_first)
        if kinds is not None:
            for st, kd in zip(sched, kinds):
                st["kind"] = kd
    X = A / alpha
    for st in sched:
        if zolo_r:
            X = zolo_step(X, st)
        else:
            step = qr_step if st["kind"] == "qr" else chol_step
            X = step(X, st["a"], st["b"], st["c"])
    B = np.eye(n) - X.T @ X
    B = 0.5 * (B + B.T)
    sub = projector_subspace(B, tol)
    out = dict(alpha=alpha, s=s, sched=sched, X=X, B=B, **sub)
    if sub["ell"] == 0:
        out.update(sigma_ritz=np.zeros(0), n_above=0)
        return out
    Q2 = sub["Q2"]
    Y = A @ Q2
    Qy, Ry = np.linalg.qr(Y, mode="reduced")
    Ut, St, Vth = np.linalg.svd(Ry)
    out.update(Qy=Qy, Ut=Ut, Vt=Vth.T, sigma_ritz=St, n_above=int(np.sum(St >= s * alpha)))
    return out


def svd_partial(A, k=None, seed=0, replay=None, s=None, tol=TOL, kappa_max=100.0,
                qr_first=None, nv=None, m=None, zolo_r=0):
    """Dominant singular triplets of A (m x n) by QDWHpartial-SVD (Algorithm 2).

    k mode: the k largest triplets.  Threshold mode (``s`` given, no k): every
    triplet with sigma >= s * alpha, alpha ~ ||A||_2, the paper's native form.
    Returns dict with U (m x k), S (descending), V (n x k) and the intermediates.
    """
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] < A.shape[1]:
        r = svd_partial(A.T, k, seed=seed, replay=replay, s=s, tol=tol,
                        kappa_max=kappa_max, qr_first=qr_first, nv=nv, m=m, zolo_r=zolo_r)
        V, U = sign_normalize(r["U"], r["V"])
        r = dict(r)
        r["U"], r["V"] = U, V
        r["transposed"] = True
        return r
    n = A.shape[1]
    kw = {} if nv is None else {"nv": nv}
    if m is not None:
        kw["m"] = m
    kinds = None if replay is None else replay.get("kinds")
    est = None
    if replay is None:
        est = lanczos_slq(lambda v: A.T @ (A @ v), n, seed, **kw)
    if k is None:
        if s is None:
            raise ValueError("give k or s")
        alpha = replay["alpha"] if replay is not None else choose_svd_threshold(est, 1)[0]
        r = _svd_core(A, alpha, s, tol, kappa_max, qr_first, kinds, zolo_r)
        k = r["n_above"]
    else:
        for boost in (1, 2):
            if replay is not None:
                alpha, sv = replay["alpha"], replay["s"]
            else:
                alpha, sv = choose_svd_threshold(est, k, boost)
            r = _svd_core(A, alpha, sv, tol, kappa_max, qr_first, kinds, zolo_r)
            if r["ell"] > 0 and (r["n_above"] >= k or r["ell"] >= n or replay is not None):
                break
        else:
            raise NoSubspace("fewer than k singular values above the threshold")
        if r["ell"] < k:
            raise NoSubspace("subspace smaller than k")
    if k == 0:
        U, S, V = np.zeros((A.shape[0], 0)), np.zeros(0), np.zeros((n, 0))
    else:
        U = r["Qy"] @ r["Ut"][:, :k]
        V = r["Q2"] @ r["Vt"][:, :k]
        S = r["sigma_ritz"][:k].copy()
        V, U = sign_normalize(V, U)
    r.update(U=U, S=S, V=V, k=k, est=est, transposed=False)
    return r
