"""Pins of the oracle's two-sided Lanczos and block-derivative method (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, estimator, matfun, tsl

DIMS = (4, 2, 2, 2)
MU = 0.3


@pytest.fixture(scope="module")
def setup():
    U = synth.make_links(DIMS, 0.5, 21)
    H = dirac.dense_h(U, DIMS, MU)
    dH = dirac.dense_dh_dmu(U, DIMS, MU)
    b = synth.make_source(DIMS, 22).ravel()
    return U, H, dH, b


def _ops(U, mu=MU):
    h = lambda v: dirac.flat(dirac.apply_h(U, v, DIMS, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, DIMS, mu))
    dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, mu))
    dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, -mu))
    return h, hd, dh, dhd


def test_full_krylov_is_exact(rng):
    """k = n: the Krylov space is the whole space and the Ritz result is exact."""
    n = 24
    lam = rng.uniform(0.5, 2.0, n) * rng.choice([-1, 1], n) + 0.2j * rng.standard_normal(n)
    S = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y, _ = tsl.krylov_sign(lambda v: A @ v, lambda v: A.conj().T @ v, b, b, n)
    ref = matfun.sign_schur(A) @ b
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-8


def test_error_falls_with_k(setup):
    U, H, dH, b = setup
    h, hd, _, _ = _ops(U)
    ref = matfun.sign_schur(H) @ b
    errs = []
    for k in (16, 32, 64, 128):
        y, _ = tsl.krylov_sign(h, hd, b, b, k)
        errs.append(np.linalg.norm(y - ref))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4


def test_relations(setup):
    """W^dag V = 1, A V = V T + r e_k^T, and the two readings of the start vectors."""
    U, H, dH, b = setup
    h, hd, _, _ = _ops(U)
    phi = synth.make_source(DIMS, 23).ravel()
    k = 20
    L = tsl.lanczos(h, hd, b, phi, k)
    V, W, T = L["V"], L["W"], L["T"]
    assert np.abs(W.conj().T @ V - np.eye(k)).max() < 1e-10
    R = H @ V - V @ T
    assert np.abs(R[:, :-1]).max() < 1e-12
    assert np.abs(H.conj().T @ W[:, :-1] - (W @ T.conj().T)[:, :-1]).max() < 1e-12
    assert np.allclose(V[:, 0], b / np.linalg.norm(b))


def test_hermitian_limit(setup):
    """mu = 0 and phi = psi: Hermitian Lanczos, T real symmetric, W = V."""
    U, _, _, b = setup
    h, hd, _, _ = _ops(U, 0.0)
    L = tsl.lanczos(h, hd, b, b, 24)
    T = L["T"]
    assert np.abs(T.imag).max() < 1e-12
    assert np.abs(T - T.T).max() < 1e-12
    assert np.abs(L["W"] - L["V"]).max() < 1e-10


def test_scalar_mode_matches_vector_mode(setup):
    U, _, _, b = setup
    h, hd, _, _ = _ops(U)
    x = synth.make_source(DIMS, 24).ravel()
    y, _ = tsl.krylov_sign(h, hd, b, b, 30)
    s, _ = tsl.krylov_sign_scalar(h, hd, b, b, 30, x)
    assert abs(s - np.vdot(x, y)) < 1e-13


def test_block_derivative_converges(setup):
    """Eq. 7 with the Krylov-Ritz method: (d sgn(H) b, sgn(H) b) approach the dense values."""
    U, H, dH, b = setup
    h, hd, dh, dhd = _ops(U)
    ref = matfun.sign_schur(H) @ b
    dref = matfun.frechet_sign_block(H, dH) @ b
    errs = []
    for k in (64, 128, 256):
        dy, y, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, k)
        errs.append(np.linalg.norm(dy - dref) / np.linalg.norm(dref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 1e-7
    assert np.linalg.norm(y - ref) < 1e-9


def test_left_start_same_fails(setup):
    """With phi = psi = (0; b) the left space never leaves (0; .): the derivative is not controlled."""
    U, H, dH, b = setup
    h, hd, dh, dhd = _ops(U)
    dref = matfun.frechet_sign_block(H, dH) @ b
    _, _, L = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, 32, rule="same")
    assert np.abs(L["W"][:b.size]).max() == 0.0
    dy_sum, _, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, 160, rule="sum")
    e_sum = np.linalg.norm(dy_sum - dref)
    try:
        dy_same, _, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, 160, rule="same")
        e_same = np.linalg.norm(dy_same - dref)
    except tsl.Breakdown:
        e_same = np.inf
    assert e_sum < 1e-3 * e_same


def test_eps_estimator(setup):
    """Sec. 4 estimate: rounding level for the dense sign, falling with k for Krylov-Ritz."""
    U, H, _, b = setup
    h, hd, _, _ = _ops(U)
    S = matfun.sign_schur(H)
    assert estimator.eps_sign(lambda v: S @ v, b) < 1e-13
    e = [estimator.eps_sign(lambda v: tsl.krylov_sign(h, hd, v, v, k)[0], b) for k in (16, 48)]
    assert e[1] < e[0] < 1


def test_breakdown_detected(rng):
    """A left start orthogonal to the right start is a serious breakdown at step 0."""
    n = 10
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = np.zeros(n, complex)
    b[0] = 1
    phi = np.zeros(n, complex)
    phi[1] = 1
    with pytest.raises((tsl.Breakdown, ZeroDivisionError, FloatingPointError, ValueError)):
        with np.errstate(all="raise"):
            tsl.lanczos(lambda v: A @ v, lambda v: A.conj().T @ v, b, phi, 5)
