"""Pins of the oracle's complex Hermitian path (oracle.hermitian) against the
real path, planted complex spectra, LAPACK's Hermitian solver and the scalar
DWH map."""
import numpy as np
import pytest

from oracle import eig_partial
from oracle.dwh import dwh_weights, dwh_map
from oracle.hermitian import heig_partial, heig_metrics, qr_step_h, chol_step_h, phase_normalize
from synthetic import eig_uniform, heig_uniform, heig_clustered, haar_complex, rng


def test_real_input_gives_the_real_result():
    A, lam = eig_uniform(200, 61)
    r = eig_partial(A, fraction=0.1, tol=0.05)
    h = heig_partial(A.astype(np.complex128), fraction=0.1, tol=0.05)
    assert h["k"] == r["k"] and h["ell"] == r["ell"] and abs(h["tau"] - r["tau"]) < 1e-12
    assert np.max(np.abs(h["w"] - r["w"])) < 1e-13
    # same vectors up to the phase convention (real sign rule vs unit-modulus rule)
    assert np.max(np.abs(np.abs(h["V"]) - np.abs(r["V"]))) < 1e-10
    assert np.max(np.abs(h["V"].imag)) < 1e-10


@pytest.mark.parametrize("n,f,which,gen", [(240, 0.1, "largest", heig_uniform), (300, 0.2, "smallest", heig_uniform),
                                           (320, 0.05, "largest", heig_clustered)])
def test_planted_complex_spectra(n, f, which, gen):
    A, lam = gen(n, 62)
    assert np.abs(A - A.conj().T).max() == 0.0 and np.abs(A.imag).max() > 0.05
    h = heig_partial(A, fraction=f, which=which, tol=0.05)
    k = h["k"]
    exact = (np.sort(lam)[::-1] if which == "largest" else np.sort(lam))[:k]
    met = heig_metrics(A, h["w"], h["V"], exact)
    assert met["value_rel_max"] < 1e-12 and met["residual"] < 1e-13 and met["orth"] < 1e-12
    ref = np.linalg.eigvalsh(A)
    ref = (ref[::-1] if which == "largest" else ref)[:k]
    assert np.max(np.abs(h["w"] - ref) / np.abs(ref)) < 1e-12
    # phase rule: the largest-magnitude entry of each vector is real positive
    idx = np.argmax(np.abs(h["V"]), axis=0)
    piv = h["V"][idx, np.arange(k)]
    assert np.all(piv.real > 0) and np.max(np.abs(piv.imag)) < 1e-15


@pytest.mark.parametrize("step", [qr_step_h, chol_step_h])
def test_complex_step_on_planted_iterate(step):
    g = rng(63)
    U = haar_complex(g, 60)[:, :40]
    V = haar_complex(g, 40)
    sig = np.geomspace(1e-3, 1.0, 40)
    X = (U * sig) @ V.conj().T
    a, b, c = dwh_weights(1e-3)
    Xn = step(X, a, b, c)
    assert np.abs(Xn - (U * dwh_map(sig, a, b, c)) @ V.conj().T).max() < 1e-12


def test_phase_normalize():
    g = rng(64)
    V = g.standard_normal((30, 5)) + 1j * g.standard_normal((30, 5))
    W = phase_normalize(V)
    assert np.allclose(np.abs(W), np.abs(V))
    idx = np.argmax(np.abs(W), axis=0)
    assert np.allclose(W[idx, np.arange(5)].imag, 0.0) and np.all(W[idx, np.arange(5)].real > 0)
