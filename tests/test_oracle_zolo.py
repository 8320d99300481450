"""Pins of the oracle's Zolotarev layer (oracle.zolo) against mathematics
independent of it: the DWH closed form (r = 1), the composition property of
Zolotarev's functions, equioscillation, and planted iterates."""
import numpy as np
import pytest

from oracle.dwh import dwh_weights, dwh_map, next_l, U_ROUND
from oracle.zolo import zolo_coeffs, zolo_map, zolo_schedule, zolo_step
from oracle.polar import chol_step, qr_step


@pytest.mark.parametrize("l", [1e-12, 1e-6, 1e-3, 0.05, 0.2, 0.5, 0.875, 0.99])
def test_r1_is_the_dwh_map(l):
    """Type (3,2): M x (x^2 + c2)/(x^2 + c1) = x (a + b x^2)/(1 + c x^2) with
    a = M c2/c1, b = M/c1, c = 1/c1 (Sec. 3.1's closed form, a different
    formula: algebraic in l instead of elliptic functions)."""
    co = zolo_coeffs(l, 1)
    c1, c2 = co["c"]
    a, b, c = dwh_weights(l)
    got = (co["M"] * c2 / c1, co["M"] / c1, 1.0 / c1)
    rel = 1e-13 if l >= 1e-3 else 1e-9      # the DWH closed form loses digits as l -> 0
    for g, w in zip(got, (a, b, c)):
        assert abs(g - w) <= rel * abs(w)
    assert abs(co["l_next"] - next_l(l, a, b, c)) <= 1e-13


@pytest.mark.parametrize("l", [1e-8, 0.01, 0.2, 0.6])
def test_composition(l):
    """Z_{(2r+1)(2r'+1)}(x; l) = Z_{2r'+1}(Z_{2r+1}(x; l); Z_{2r+1}(l; l)): the
    DWH map applied twice is type (9,8) (r = 4), three times type (27,26)
    (r = 13) -- the three DWH steps from s = 0.2 of Sec. 4.1 are one
    Zolotarev step of type (27,26)."""
    x = np.concatenate([np.geomspace(l, 1.0, 2001), np.linspace(l, 1.0, 2001)])
    y, lk = x.copy(), l
    for steps, r in ((2, 4), (3, 13)):
        y, lk = x.copy(), l
        for _ in range(steps):
            w = dwh_weights(lk)
            y = dwh_map(y, *w)
            lk = next_l(lk, *w)
        co = zolo_coeffs(l, r)
        tol = 1e-12 if l >= 0.01 else 1e-9
        assert np.abs(zolo_map(x, co) - y).max() <= tol
        assert abs(co["l_next"] - lk) <= tol


@pytest.mark.parametrize("l,r", [(0.2, 2), (0.2, 3), (0.05, 4), (0.01, 5)])
def test_equioscillation(l, r):
    """On [l, 1] Z stays within [Z(l), 1], reaching 1 at r + 1 points (x = 1
    among them) and Z(l) at r + 1 points (x = l among them): the 2r + 2
    alternation points of the best approximation."""
    co = zolo_coeffs(l, r)
    x = np.linspace(l, 1.0, 400001)
    z = zolo_map(x, co)
    lo = co["l_next"]
    assert z.max() <= 1.0 + 8 * U_ROUND and z.min() >= lo * (1 - 1e-13)
    assert abs(z[-1] - 1.0) < 8 * U_ROUND and abs(z[0] - lo) < 1e-15
    interior = (z[1:-1] >= z[:-2]) & (z[1:-1] >= z[2:])
    peaks = np.nonzero(interior)[0] + 1
    troughs = np.nonzero((z[1:-1] <= z[:-2]) & (z[1:-1] <= z[2:]))[0] + 1
    assert len(peaks) == r and np.all(np.abs(z[peaks] - 1.0) < 1e-9)
    assert len(troughs) == r and np.all(np.abs(z[troughs] - lo) < 1e-9 * max(1.0, lo))


def test_partial_fractions_reproduce_the_product():
    for l, r in ((0.2, 2), (1e-4, 6), (0.7, 3)):
        co = zolo_coeffs(l, r)
        y = np.geomspace(1e-6, 1e3, 500)
        prod = np.ones_like(y)
        pf = np.ones_like(y)
        for j in range(r):
            prod *= (y + co["c"][2 * j + 1]) / (y + co["c"][2 * j])
            pf += co["a"][j] / (y + co["c"][2 * j])
        assert np.abs(pf - prod).max() <= 1e-12 * np.abs(prod).max()


def test_increasing_beyond_one():
    """x+ = max(1, Z(x)) bounds the unwanted side only if Z >= 1 and does not
    decrease on [1, inf) (it is flat to rounding next to 1 when the
    approximation error is below u)."""
    for l, r in ((0.2, 2), (0.2, 13), (1e-6, 8)):
        co = zolo_coeffs(l, r)
        x = np.linspace(1.0, 50.0, 20001)
        z = zolo_map(x, co)
        assert np.all(z >= 1.0 - 4 * U_ROUND) and np.all(np.diff(z) >= -4 * U_ROUND)
        assert z[-1] > 2.0


def _planted(m, n, sig, seed):
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((m, n)))
    V, _ = np.linalg.qr(g.standard_normal((n, n)))
    return (U * sig) @ V.T, U, V


@pytest.mark.parametrize("kind", ["chol", "qr"])
def test_step_on_planted_iterate(kind):
    sig = np.geomspace(0.2, 1.0, 40)
    X, U, V = _planted(70, 40, sig, 3)
    co = zolo_coeffs(0.2, 3)
    st = dict(co=co, kinds=[kind] * 3)
    Xn = zolo_step(X, st)
    assert np.abs(Xn - (U * zolo_map(sig, co)) @ V.T).max() < 1e-13


def test_r1_step_is_the_dwh_step():
    sig = np.geomspace(1e-3, 1.0, 30)
    X, _, _ = _planted(50, 30, sig, 4)
    co = zolo_coeffs(1e-3, 1)
    a, b, c = dwh_weights(1e-3)
    for kind, ref in (("qr", qr_step(X, a, b, c)), ("chol", chol_step(X, a, b, c))):
        assert np.abs(zolo_step(X, dict(co=co, kinds=[kind])) - ref).max() < 1e-12


def test_schedule_steps_and_kinds():
    # s = 0.2: one step of type (27,26) reaches |l - 1| < 5u; type (5,4) two
    assert len(zolo_schedule(0.2, 13)) == 1
    assert len(zolo_schedule(0.2, 2)) == 2
    assert len(zolo_schedule(0.2, 1)) == 3          # = the three DWH steps of Sec. 4.1
    # terms with small c_{2j-1} need the QR form once the bound exceeds kappa_max
    st = zolo_schedule(0.2, 4)[0]
    assert st["kinds"][0] == "qr" and st["kinds"][-1] == "chol"
    assert all(k == "chol" for k in zolo_schedule(0.2, 2)[0]["kinds"])
    sv = zolo_schedule(1e-12, 8, qr_first=True)
    assert len(sv) == 2 and all(k == "qr" for k in sv[0]["kinds"])


def test_partial_eig_and_svd_with_zolotarev_steps():
    """Algorithms 1 and 2 with Zolotarev steps reach the planted spectra."""
    from oracle import eig_partial, svd_partial, eig_metrics, svd_metrics
    from synthetic import eig_uniform, svd_geometric
    A, lam = eig_uniform(300, 71)
    for r in (1, 2, 13):
        out = eig_partial(A, fraction=0.1, zolo_r=r, tol=0.05)
        k = out["k"]
        exact = np.sort(lam)[::-1][:k]
        assert np.max(np.abs(out["w"] - exact) / np.abs(exact)) < 1e-12
        assert eig_metrics(A, out["w"], out["V"], exact)["residual"] < 1e-13
    dwh = eig_partial(A, fraction=0.1, zolo_r=0, tau_policy="plain", tol=0.05)
    z1 = eig_partial(A, fraction=0.1, zolo_r=1, tol=0.05)
    assert z1["ell"] == dwh["ell"] and np.abs(z1["X"] - dwh["X"]).max() < 1e-12
    A, sig = svd_geometric(260, 200, 72, kappa=1e16)
    for r in (2, 8):
        out = svd_partial(A, 12, zolo_r=r, tol=0.05, qr_first=True)
        assert len(out["sched"]) <= 3
        assert np.max(np.abs(out["S"] - sig[:12]) / sig[:12]) < 1e-12
        assert svd_metrics(A, out["U"], out["S"], out["V"], sig[:12])["residual"] < 1e-13
