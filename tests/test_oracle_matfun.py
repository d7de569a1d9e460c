"""Pins of the oracle's dense matrix sign and its derivative (no GPU)."""
import numpy as np
import pytest

from oracle import matfun


def _random_split_matrix(rng, n, gap=0.5):
    """Random non-normal matrix with eigenvalues away from the imaginary axis."""
    lam = rng.uniform(gap, 3.0, n) * rng.choice([-1, 1], n) + 0.4j * rng.standard_normal(n)
    S = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * np.eye(n)
    return S @ np.diag(lam) @ np.linalg.inv(S), lam


def test_scalar_and_diagonal():
    d = np.array([2.0 + 1j, -0.5 + 3j, 0.1 - 0.2j, -4.0])
    for f in (matfun.sign_eig, matfun.sign_schur, matfun.sign_newton):
        assert np.allclose(f(np.diag(d)), np.diag([1, -1, 1, -1]), atol=1e-13)


def test_three_methods_agree(rng):
    A, _ = _random_split_matrix(rng, 24)
    S1, S2, S3 = matfun.sign_eig(A), matfun.sign_schur(A), matfun.sign_newton(A)
    assert np.abs(S1 - S2).max() < 1e-11
    assert np.abs(S3 - S2).max() < 1e-11
    assert np.abs(S2 @ S2 - np.eye(24)).max() < 1e-11
    assert np.abs(S2 @ A - A @ S2).max() < 1e-10


def test_hermitian_textbook(rng):
    Z = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    A = Z + Z.conj().T
    w, Q = np.linalg.eigh(A)
    ref = (Q * np.sign(w)) @ Q.conj().T
    assert np.abs(matfun.sign_schur(A) - ref).max() < 1e-12


def test_jordan_block_sign():
    """Eq. 5 for sgn: f' = 0 off the imaginary axis, so sgn(J) = sgn(lambda) I."""
    for lam in (0.7 + 0.2j, -1.3 + 0.1j):
        J = np.array([[lam, 1.0], [0.0, lam]])
        s = 1.0 if lam.real > 0 else -1.0
        assert np.allclose(matfun.sign_schur(J), s * np.eye(2), atol=1e-14)
        assert np.allclose(matfun.sign_newton(J), s * np.eye(2), atol=1e-12)


def test_block_identity_against_divided_differences(rng):
    """Eq. 6: top-right block of sgn([[A, E], [0, A]]) is the Frechet derivative."""
    A, _ = _random_split_matrix(rng, 20)
    E = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    L1 = matfun.frechet_sign_block(A, E)
    L2 = matfun.frechet_sign_dd(A, E)
    L3 = matfun.frechet_sign_block(A, E, matfun.sign_newton)
    assert np.abs(L1 - L2).max() < 1e-10 * max(1, np.abs(L2).max())
    assert np.abs(L1 - L3).max() < 1e-10 * max(1, np.abs(L2).max())
    # diagonal blocks are sgn(A)
    B = matfun.sign_schur(matfun.block(A, E))
    assert np.abs(B[:20, :20] - matfun.sign_schur(A)).max() < 1e-11
    assert np.abs(B[20:, :20]).max() < 1e-12


def test_block_identity_finite_difference(rng):
    A, _ = _random_split_matrix(rng, 12)
    E = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    h = 1e-6
    fd = (matfun.sign_schur(A + h * E) - matfun.sign_schur(A - h * E)) / (2 * h)
    L = matfun.frechet_sign_block(A, E)
    assert np.abs(fd - L).max() < 1e-6 * max(1, np.abs(L).max())


def test_derivative_anticommutes(rng):
    """d(S^2) = 0  =>  S dS + dS S = 0."""
    A, _ = _random_split_matrix(rng, 16)
    E = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    S = matfun.sign_schur(A)
    L = matfun.frechet_sign_block(A, E)
    assert np.abs(S @ L + L @ S).max() < 1e-10 * max(1, np.abs(L).max())
