"""Zolotarev higher-order steps: the variant named beside the DWH iteration
(Sec. 3.1, closing remarks; Sec. 9, future work: higher-order rational
functions).  Test infrastructure only: nothing in the library imports it.

Zolotarev's best rational approximation of type (2r+1, 2r) to sign(x) on
[-1, -l] u [l, 1], scaled to have its maximum 1 on [l, 1] (r = 1 is the DWH
map of Sec. 3.1), as given by Nakatsukasa and Freund (SIAM Review 58, 2016,
"Computing fundamental matrix decompositions accurately via the matrix sign
function in two iterations: the power of Zolotarev's functions"):

    Z(x) = M x prod_{j=1..r} (x^2 + c_{2j}) / (x^2 + c_{2j-1}),
    c_i  = l^2 sn^2(i K'/(2r+1); l') / cn^2(i K'/(2r+1); l'),  i = 1 .. 2r,
    l'   = sqrt(1 - l^2),  K' = K(l'),
    M    = prod_j (1 + c_{2j-1}) / (1 + c_{2j})      (so that Z(1) = 1),

and the next lower bound is l+ = Z(l).  In y = x^2 the product has the
partial fractions 1 + sum_j a_j / (y + c_{2j-1}) with
a_j = prod_k (c_{2k} - c_{2j-1}) / prod_{k != j} (c_{2k-1} - c_{2j-1}), so
one step is

    X+ = M (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1}),

each term by a Cholesky factorization of X^T X + c I or, when that is ill
conditioned, by the QR factorization [X / sqrt(c); I] = [Q1; Q2] R, which
gives X (X^T X + c I)^{-1} = Q1 Q2^T / sqrt(c).

The elliptic functions come from mpmath at 80 significant digits (library
routines serving as steps).

Readings (the paper gives no schedule for these steps):
  * steps from l_0 until |l_k - 1| < 5u, as the SVD's DWH schedule;
  * a term is QR-based when its bound 1 + x^2 / c_{2j-1} on the condition
    number of I + X^T X / c_{2j-1} exceeds kappa_max (x = 1 for the SVD, the
    bound on the largest unwanted scaled eigenvalue for the EIG, updated as
    x+ = max(1, Z(x))); the same rule as the DWH steps, which it reduces to
    at r = 1; qr_first forces every term of the first step QR-based;
  * the EIG threshold takes the plain cut (the cost model is the DWH one).
"""
import math

import mpmath as mp
import numpy as np
import scipy.linalg as sla

from .dwh import U_ROUND

_DPS = 80


def zolo_coeffs(l, r):
    """c_1 .. c_2r, a_1 .. a_r, M and l+ = Z(l) for lower bound l in (0, 1)."""
    if not (0.0 < l < 1.0) or r < 1:
        raise ValueError("need 0 < l < 1 and r >= 1")
    with mp.workdps(_DPS):
        L = mp.mpf(l)
        m = 1 - L * L                        # parameter of the modulus l'
        Kp = mp.ellipk(m)
        c = []
        for i in range(1, 2 * r + 1):
            u = i * Kp / (2 * r + 1)
            sn = mp.ellipfun("sn", u, m=m)
            cn = mp.ellipfun("cn", u, m=m)
            c.append(L * L * sn * sn / (cn * cn))
        M = mp.mpf(1)
        for j in range(r):
            M *= (1 + c[2 * j]) / (1 + c[2 * j + 1])
        a = []
        for j in range(r):
            num = mp.mpf(1)
            for k in range(r):
                num *= c[2 * k + 1] - c[2 * j]
            den = mp.mpf(1)
            for k in range(r):
                if k != j:
                    den *= c[2 * k] - c[2 * j]
            a.append(num / den)
        lz = M * L
        for j in range(r):
            lz *= (L * L + c[2 * j + 1]) / (L * L + c[2 * j])
        return dict(r=r, c=[float(v) for v in c], a=[float(v) for v in a], M=float(M),
                    l_next=min(float(lz), 1.0))


def zolo_map(x, co):
    """Z(x) in product form, elementwise for arrays."""
    x = np.asarray(x, dtype=np.float64)
    y = x * x
    z = co["M"] * x
    for j in range(co["r"]):
        z = z * (y + co["c"][2 * j + 1]) / (y + co["c"][2 * j])
    return z


def zolo_schedule(s, r, kappa_max=100.0, x0=1.0, qr_first=False, max_iter=8):
    """Steps from l_0 = s until |l_k - 1| < 5u; per step the coefficients,
    the kinds of its r terms ('qr' | 'chol'), l_k and the bound x_k."""
    sched = []
    l, x = float(s), float(x0)
    while abs(l - 1.0) >= 5.0 * U_ROUND and len(sched) < max_iter:
        co = zolo_coeffs(min(l, 1.0 - 1e-16), r)
        kinds = []
        for j in range(r):
            force = qr_first and not sched
            kinds.append("qr" if force or 1.0 + x * x / co["c"][2 * j] > kappa_max else "chol")
        sched.append(dict(co=co, kinds=kinds, l=l, x=x,
                          kind="qr" if "qr" in kinds else "chol"))
        l = co["l_next"]
        x = max(1.0, float(zolo_map(x, co)))
    return sched


def _term_chol(X, c):
    """X (X^T X + c I)^{-1} by the upper Cholesky factor W of X^T X + c I:
    two triangular solves, as Eq. (3)."""
    n = X.shape[1]
    W = sla.cholesky(X.T @ X + c * np.eye(n), lower=False)
    Y1t = sla.solve_triangular(W, X.T, trans="T", lower=False)
    return sla.solve_triangular(W, Y1t, trans="N", lower=False).T


def _term_qr(X, c):
    """X (X^T X + c I)^{-1} = Q1 Q2^T / sqrt(c) from [X / sqrt(c); I] = [Q1; Q2] R."""
    m, n = X.shape
    Q, _ = np.linalg.qr(np.vstack([X / math.sqrt(c), np.eye(n)]), mode="reduced")
    return (Q[:m] @ Q[m:].T) / math.sqrt(c)


def zolo_step(X, st):
    """One step X+ = M (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1})."""
    co = st["co"]
    acc = X.copy()
    for j in range(co["r"]):
        cj = co["c"][2 * j]
        term = _term_qr(X, cj) if st["kinds"][j] == "qr" else _term_chol(X, cj)
        acc = acc + co["a"][j] * term
    return co["M"] * acc
