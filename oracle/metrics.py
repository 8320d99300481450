"""Accuracy metrics for partial results (Sec. 7.3, with readings).

Sec. 7.3 defines orthogonality ||I - U U^T||_F / n, value accuracy
||Sigma - Delta||_F / ||Delta||_F and residuals max_i ||A v_i - sigma_i u_i||.
For k < n the first is not small for a partial basis and the residuals carry
no normalisation, so the reading used here is: orthogonality ||I_k - V^T V||_F;
residual max_i ||A v_i - lambda_i v_i||_2 / ||A||_2 (SVD: the larger of the two
one-sided residuals); values both normwise (as printed) and as the maximum
per-value relative error against the exact (planted) values.
"""
import numpy as np


def _norm2(A):
    return float(np.linalg.norm(A, 2)) if min(A.shape) <= 2048 else float(
        np.sqrt(np.max(np.linalg.eigvalsh(A.T @ A))))


def eig_metrics(A, w, V, exact=None, anorm=None):
    anorm = _norm2(A) if anorm is None else anorm
    R = A @ V - V * w[None, :]
    out = dict(
        residual=float(np.max(np.linalg.norm(R, axis=0))) / anorm,
        residual_fro=float(np.sqrt(2.0) * np.linalg.norm(R) / np.linalg.norm(A)),
        orth=float(np.linalg.norm(np.eye(V.shape[1]) - V.T @ V)),
    )
    if exact is not None:
        out["value_rel_max"] = float(np.max(np.abs(w - exact) / np.abs(exact)))
        out["value_rel_fro"] = float(np.linalg.norm(w - exact) / np.linalg.norm(exact))
    return out


def svd_metrics(A, U, S, V, exact=None, anorm=None):
    anorm = _norm2(A) if anorm is None else anorm
    r1 = np.linalg.norm(A @ V - U * S[None, :], axis=0)
    r2 = np.linalg.norm(A.T @ U - V * S[None, :], axis=0)
    out = dict(
        residual=float(max(np.max(r1), np.max(r2))) / anorm,
        orth_u=float(np.linalg.norm(np.eye(U.shape[1]) - U.T @ U)),
        orth_v=float(np.linalg.norm(np.eye(V.shape[1]) - V.T @ V)),
    )
    if exact is not None:
        out["value_rel_max"] = float(np.max(np.abs(S - exact) / np.abs(exact)))
        out["value_rel_fro"] = float(np.linalg.norm(S - exact) / np.linalg.norm(exact))
    return out
