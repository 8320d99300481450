"""Scalar layer of the dynamically weighted Halley (DWH) iteration.

Sec. 3.1: the weights (a_k, b_k, c_k) make r_k(x) = x (a_k + b_k x^2)/(1 + c_k x^2)
the scaled Zolotarev (3,2) best approximation to sign(x) on [-1,-l_k] u [l_k,1],
and l_{k+1} = r_k(l_k).  The closed form of the weights is the one written out
in Algorithm 3 (Sec. 5).

Readings where the paper is silent or garbled:
  * the parenthesis of the square root in the weight formula of Algorithm 3 is
    unbalanced; it is read as a = sqd + sqrt(8 - 4 dd + 8 (2 - l^2)/(l^2 sqd))/2,
    which is the reading for which r has the equioscillation property (pinned
    in the tests);
  * l is clamped to at most 1 before the weights are formed: rounding can push
    l_k to 1 + O(u), where the cube root of a negative number has no real
    value; l = 1 gives Halley's weights (3, 1, 3);
  * "5eps" / "O(u)" in the stopping rule |l_k - 1| < 5 eps is read with
    eps = u = 2^-53.
"""
import math

U_ROUND = 2.0 ** -53   # unit roundoff of IEEE double


def dwh_weights(l):
    """(a, b, c) for lower bound l in (0, 1] (Sec. 3.1; closed form of Algorithm 3)."""
    l = min(float(l), 1.0)
    if not (l > 0.0):
        raise ValueError("DWH lower bound must be positive")
    l2 = l * l
    dd = (4.0 * (1.0 - l2) / (l2 * l2)) ** (1.0 / 3.0)
    sqd = math.sqrt(1.0 + dd)
    a = sqd + 0.5 * math.sqrt(8.0 - 4.0 * dd + 8.0 * (2.0 - l2) / (l2 * sqd))
    b = (a - 1.0) ** 2 / 4.0
    c = a + b - 1.0
    return a, b, c


def dwh_map(x, a, b, c):
    """r(x) = x (a + b x^2) / (1 + c x^2) (Sec. 3.1), elementwise for arrays."""
    x2 = x * x
    return x * (a + b * x2) / (1.0 + c * x2)


def compose(x, weights):
    """r_K(... r_1(x)) for a list of (a, b, c) weights: the scalar image of the
    singular values (Sec. 3.1: the composite maps Sigma to r_k(...r_1(Sigma)))."""
    for (a, b, c) in weights:
        x = dwh_map(x, a, b, c)
    return x


def next_l(l, a, b, c):
    """l_{k+1} = r_k(l_k) (Sec. 3.1)."""
    return dwh_map(min(l, 1.0), a, b, c)


def iteration_count(l0, max_iter=12):
    """Number of iterations until |l_k - 1| < 5u (Sec. 4.2 stopping rule)."""
    l = float(l0)
    k = 0
    while abs(l - 1.0) >= 5.0 * U_ROUND and k < max_iter:
        a, b, c = dwh_weights(l)
        l = next_l(l, a, b, c)
        k += 1
    return k


QR_FIRST_BELOW = 1e-3   # Sec. 4.2: QR-based first step when s << 1 ("say s < 1e-3")


def svd_schedule(s, kappa_max=100.0, qr_first=None, max_iter=12):
    """Weights and kinds for QDWHpartial-SVD (Algorithm 2): start from l_0 = s,
    stop at |l_k - 1| < 5u.

    Kind of each step: Sec. 4.2 advises the QR-based Eq. (2) for the first
    iteration when s << 1 (s < 1e-3); Cholesky-based Eq. (3) steps are safe
    once Z_k = I + c_k X_k^T X_k is well conditioned (Sec. 3.1), and since
    the singular values of X_k lie in [0, 1], 1 + c_k bounds cond(Z_k).
    Reading: a step is QR-based while 1 + c_k exceeds ``kappa_max`` (which
    covers the s < 1e-3 rule: c_0 > 1.6e4 there), Cholesky-based otherwise.
    ``qr_first`` None follows that rule; True forces step 0 to be QR-based
    (Table 1 counts one QR-based iteration for the SVD); False never forces it.
    Returns a list of dicts with keys a, b, c, kind ('qr'|'chol'), l (l_k before the step).
    """
    force = (float(s) < QR_FIRST_BELOW) if qr_first is None else bool(qr_first)
    sched = []
    l = float(s)
    while abs(l - 1.0) >= 5.0 * U_ROUND and len(sched) < max_iter:
        a, b, c = dwh_weights(l)
        kappa = 1.0 + c
        kind = "qr" if ((force and not sched) or kappa > kappa_max) else "chol"
        sched.append(dict(a=a, b=b, c=c, kind=kind, l=l))
        l = next_l(l, a, b, c)
    return sched


def eig_schedule(s, rho, iters=3, kappa_max=100.0):
    """Weights and kinds for QDWHpartial-EIG (Algorithm 1): ``iters`` steps from l_0 = s.

    ``rho`` bounds the largest unwanted eigenvalue of the scaled matrix
    (tau - lambda_min)/|mu|, so the largest singular value of
    X_0 = (1-s) B - s I is x_0 = max(1, (1-s) rho - s); thereafter
    x_{k+1} = max(1, r_k(x_k)) because r_k <= 1 on [l_k, 1] and r_k is
    increasing on [1, inf).  Reading (Sec. 4.1 says Cholesky is safe in all
    iterations when the spectrum lies in [-1, 1]): a step is QR-based when the
    bound 1 + c_k x_k^2 on cond(Z_k) exceeds ``kappa_max``, Cholesky-based
    otherwise.
    """
    sched = []
    l = float(s)
    x = max(1.0, (1.0 - s) * float(rho) - s)
    for _ in range(iters):
        a, b, c = dwh_weights(l)
        kappa = 1.0 + c * x * x
        sched.append(dict(a=a, b=b, c=c, kind="qr" if kappa > kappa_max else "chol",
                          l=l, x=x))
        l = next_l(l, a, b, c)
        x = max(1.0, dwh_map(x, a, b, c))
    return sched
