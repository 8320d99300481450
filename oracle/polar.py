"""One dynamically weighted Halley step in the paper's three forms (Sec. 3.1).

  Eq. (1)  X+ = X (a I + b X^T X) (I + c X^T X)^{-1}                 (direct)
  Eq. (2)  [sqrt(c) X; I] = [Q1; Q2] R,
           X+ = (b/c) X + (a - b/c)/sqrt(c) Q1 Q2^T                  (QR-based)
  Eq. (3)  Z = I + c X^T X, W = chol(Z),
           X+ = (b/c) X + (a - b/c) (X W^{-1}) W^{-T}                (Cholesky-based)

The solver uses Eq. (2) and Eq. (3); Eq. (1) is kept only as an independent
cross-check in the tests.  LAPACK's Householder QR and Cholesky serve as
library steps.
"""
import numpy as np
import scipy.linalg as sla


def qr_step(X, a, b, c):
    """Eq. (2): QR-based step on the stacked (m+n) x n matrix [sqrt(c) X; I]."""
    m, n = X.shape
    W = np.vstack([np.sqrt(c) * X, np.eye(n)])
    Q, _ = np.linalg.qr(W, mode="reduced")
    Q1, Q2 = Q[:m], Q[m:]
    return (b / c) * X + (a - b / c) / np.sqrt(c) * (Q1 @ Q2.T)


def chol_step(X, a, b, c):
    """Eq. (3): Cholesky-based step; W is the upper Cholesky factor of Z = W^T W."""
    n = X.shape[1]
    Z = np.eye(n) + c * (X.T @ X)
    W = sla.cholesky(Z, lower=False)
    # (X W^{-1}) W^{-T}: two right-side triangular solves, written as solves
    # with the transposed systems W^T Y1^T = X^T and W Y^T = Y1^T.
    Y1t = sla.solve_triangular(W, X.T, trans="T", lower=False)
    Yt = sla.solve_triangular(W, Y1t, trans="N", lower=False)
    return (b / c) * X + (a - b / c) * Yt.T


def halley_direct_step(X, a, b, c):
    """Eq. (1) with an explicit inverse: a cross-check only, never used by the solver."""
    n = X.shape[1]
    G = X.T @ X
    return X @ (a * np.eye(n) + b * G) @ np.linalg.inv(np.eye(n) + c * G)
