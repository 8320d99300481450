"""Readings behind the exact split of large EIG Rayleigh-Ritz matrices,
checked on the CPU in FP64 numpy (no GPU code is involved).

The split takes the polar factor of (H - sigma I) / alpha to convergence with
the Sec. 3.1 schedule from l0 = 1e-12; its QR-form steps take the QR of the
stacked [sqrt(c) X; I] by shifted Cholesky QR in three rounds (a Gram shifted
by 11 (2n^2 + n(n+1)) u (c + 1), then two plain rounds) instead of Householder
QR.  These tests pin that substitution against the oracle's Eq. (2) step
(LAPACK Householder QR) and against the exact sign function, and check that
C = (I + X) / 2 then counts the eigenvalues above the shift."""
import math

import numpy as np
import pytest

from oracle.dwh import svd_schedule
from oracle.polar import chol_step, qr_step

U = 2.0 ** -53


def _cholqr3_step(X, a, b, c):
    """The QR-form step with the QR of W = [sqrt(c) X; I] by shifted Cholesky
    QR in three rounds (the reading under test, written out in numpy)."""
    n = X.shape[0]
    src = np.vstack([math.sqrt(c) * X, np.eye(n)])
    for rnd in range(3):
        G = src.T @ src
        if rnd == 0:
            G = G + 11.0 * (2 * n * n + n * (n + 1)) * U * (c + 1.0) * np.eye(n)
        R = np.linalg.cholesky(G).T
        src = np.linalg.solve(R.T, src.T).T          # src R^{-1}
    Xn = (b / c) * X + (a - b / c) / math.sqrt(c) * (src[:n] @ src[n:].T)
    return 0.5 * (Xn + Xn.T), src


def _planted(n, seed, tiny):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    half = (n - len(tiny)) // 2
    lam = np.concatenate([g.uniform(-0.95, -1e-3, half), g.uniform(1e-3, 0.95, n - len(tiny) - half), tiny])
    X = (Q * lam) @ Q.T
    return 0.5 * (X + X.T), Q, lam


@pytest.mark.parametrize("seed", [0, 1])
def test_cholesky_qr_steps_reach_the_sign_function(seed):
    n = 160
    X0, Q, lam = _planted(n, seed, np.array([3e-11, -7e-11]))
    sched = svd_schedule(1e-12, kappa_max=100.0, qr_first=False)
    assert [s["kind"] for s in sched] == ["qr", "qr", "chol", "chol", "chol"]
    Xh, Xc = X0.copy(), X0.copy()
    for st in sched:
        a, b, c = st["a"], st["b"], st["c"]
        if st["kind"] == "qr":
            Xh = qr_step(Xh, a, b, c)
            Xh = 0.5 * (Xh + Xh.T)
            Xc, Qc = _cholqr3_step(Xc, a, b, c)
            # the three rounds leave Q orthonormal to working accuracy even at
            # c ~ 1.6e16 (cond(W) ~ 1e8, beyond plain two-round Cholesky QR)
            assert np.abs(Qc.T @ Qc - np.eye(n)).max() < 50 * n * U
        else:
            Xh = chol_step(Xh, a, b, c)
            Xc = chol_step(Xc, a, b, c)
            Xh, Xc = 0.5 * (Xh + Xh.T), 0.5 * (Xc + Xc.T)
    S = (Q * np.sign(lam)) @ Q.T
    # on the eigenvectors of the separated eigenvalues (|lambda| >= 1e-3)
    # both forms give the sign function to working accuracy; the two tiny
    # eigenvalues' directions carry the rounding of X0 amplified by
    # 1/|lambda| (about u / 3e-11) in either form
    P = Q[:, np.abs(lam) >= 1e-3]
    assert np.abs(P.T @ (Xc - S) @ P).max() < 1e-13
    assert np.abs(P.T @ (Xh - S) @ P).max() < 1e-13
    assert np.abs(Xc - S).max() < 1e-6 and np.abs(Xh - S).max() < 1e-6


def test_cholesky_qr_orthogonality_at_large_size():
    """The first QR-form step from l0 = 1e-12 (c ~ 1.6e16, cond(W) ~ 1.3e8)
    at a size where the proved range of shifted Cholesky QR ends below that
    condition number: Q must still come out orthonormal to working accuracy."""
    n = 2048
    g = np.random.default_rng(11)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.concatenate([np.geomspace(1e-12, 1.0, n // 2), -np.geomspace(1e-12, 1.0, n - n // 2)])
    X = (Q * lam) @ Q.T
    X = 0.5 * (X + X.T)
    st = svd_schedule(1e-12, kappa_max=100.0, qr_first=False)[0]
    assert st["kind"] == "qr" and st["c"] > 1e16
    Xn, Qc = _cholqr3_step(X, st["a"], st["b"], st["c"])
    assert np.abs(Qc.T @ Qc - np.eye(n)).max() < 50 * n * U
    # and the step matches the oracle's Householder form of Eq. (2): to
    # working accuracy on the directions of the eigenvalues >= 1e-3, and
    # everywhere within the rounding amplification of the step itself (its
    # slope at 0 is a ~ 2.5e8, so an O(u) perturbation of X moves X+ by a u)
    Xh = qr_step(X, st["a"], st["b"], st["c"])
    Xh = 0.5 * (Xh + Xh.T)
    P = Q[:, np.abs(lam) >= 1e-3]
    assert np.abs(P.T @ (Xn - Xh) @ P).max() < 1e-12
    assert np.abs(Xn - Xh).max() < 4 * st["a"] * U


def test_projector_counts_the_eigenvalues_above_the_shift():
    n = 140
    g = np.random.default_rng(5)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.sort(g.uniform(0.1, 1.0, n))
    H = (Q * lam) @ Q.T
    sigma = 0.5 * (lam[60] + lam[61])          # 79 eigenvalues above sigma
    alpha = 1.05 * max(lam[-1] - sigma, sigma - lam[0])
    X = (H - sigma * np.eye(n)) / alpha
    l0 = min(abs(lam - sigma)) / alpha
    for st in svd_schedule(min(l0, 1e-12), kappa_max=100.0, qr_first=False):
        if st["kind"] == "qr":
            X, _ = _cholqr3_step(X, st["a"], st["b"], st["c"])
        else:
            X = chol_step(X, st["a"], st["b"], st["c"])
            X = 0.5 * (X + X.T)
    C = 0.5 * (np.eye(n) + X)
    assert round(np.trace(C)) == n - 61
    # C is the orthogonal projector onto the eigenvectors above sigma
    V = Q[:, 61:]
    assert np.abs(C - V @ V.T).max() < 1e-13
