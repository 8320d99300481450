"""Brute-force cyclic Jacobi eigen/singular value solvers for tiny matrices.

These are textbook methods (two-sided cyclic-by-row Jacobi for symmetric
matrices; one-sided Hestenes Jacobi for the SVD), written with plain Python
loops over index pairs.  They share nothing with LAPACK or with the
partial-spectrum method and serve only to pin the oracle on n <= 64.
"""
import math
import numpy as np


def _sym_schur(app, aqq, apq):
    """Rotation (c, s) that zeroes the (p, q) entry of a symmetric 2x2 block."""
    if apq == 0.0:
        return 1.0, 0.0
    d = aqq - app
    if abs(apq) < 1e-150 * abs(d):
        t = apq / d            # tau = d/(2 apq) is huge: t ~ 1/(2 tau)
    else:
        tau = d / (2.0 * apq)
        t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    return c, t * c


def jacobi_eig(A, tol=None, max_sweeps=60):
    """All eigenpairs of symmetric A, values in descending order."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    V = np.eye(n)
    fro = np.linalg.norm(A)
    tol = 2.0 ** -53 * fro if tol is None else tol
    for _ in range(max_sweeps):
        off = math.sqrt(max(0.0, np.sum(A * A) - np.sum(np.diag(A) ** 2)))
        if off <= tol:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c, s = _sym_schur(A[p, p], A[q, q], A[p, q])
                if s == 0.0:
                    continue
                Ap, Aq = A[:, p].copy(), A[:, q].copy()
                A[:, p], A[:, q] = c * Ap - s * Aq, s * Ap + c * Aq
                Ap, Aq = A[p, :].copy(), A[q, :].copy()
                A[p, :], A[q, :] = c * Ap - s * Aq, s * Ap + c * Aq
                Vp, Vq = V[:, p].copy(), V[:, q].copy()
                V[:, p], V[:, q] = c * Vp - s * Vq, s * Vp + c * Vq
    w = np.diag(A).copy()
    order = np.argsort(-w, kind="stable")
    return w[order], V[:, order]


def jacobi_svd(A, tol=1e-15, max_sweeps=60):
    """All singular triplets of A (m >= n) by one-sided Jacobi, descending."""
    G = np.array(A, dtype=np.float64)
    m, n = G.shape
    V = np.eye(n)
    for _ in range(max_sweeps):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                alpha = float(G[:, p] @ G[:, p])
                beta = float(G[:, q] @ G[:, q])
                gamma = float(G[:, p] @ G[:, q])
                if abs(gamma) <= tol * math.sqrt(alpha * beta) or gamma == 0.0:
                    continue
                rotated = True
                c, s = _sym_schur(alpha, beta, gamma)
                Gp, Gq = G[:, p].copy(), G[:, q].copy()
                G[:, p], G[:, q] = c * Gp - s * Gq, s * Gp + c * Gq
                Vp, Vq = V[:, p].copy(), V[:, q].copy()
                V[:, p], V[:, q] = c * Vp - s * Vq, s * Vp + c * Vq
        if not rotated:
            break
    S = np.sqrt(np.sum(G * G, axis=0))
    order = np.argsort(-S, kind="stable")
    S, G, V = S[order], G[:, order], V[:, order]
    U = G / np.where(S > 0, S, 1.0)[None, :]
    return U, S, V
