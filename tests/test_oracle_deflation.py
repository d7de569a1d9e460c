"""Pins of the oracle's standard and generalised deflation (no GPU)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import deflation, dirac, matfun, tsl

DIMS = (2, 2, 2, 4)
MU = 0.3


@pytest.fixture(scope="module")
def setup():
    U = synth.make_links(DIMS, 1.0, 31)   # rough links: smaller spectral gap
    H = dirac.dense_h(U, DIMS, MU)
    dH = dirac.dense_dh_dmu(U, DIMS, MU)
    b = synth.make_source(DIMS, 32).ravel()
    return U, H, dH, b


def _ops(U, mu=MU):
    h = lambda v: dirac.flat(dirac.apply_h(U, v, DIMS, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, DIMS, mu))
    dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, mu))
    dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, -mu))
    return h, hd, dh, dhd


def test_jordan_basis_of_block_matrix(rng):
    """Eq. 9-10: the analytic X, X^{-1} of B put it in Jordan form (complete set, small A)."""
    n = 6
    A0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    dA = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(A0, dA, n)
    X = np.zeros((2 * n, 2 * n), complex)
    Xi = np.zeros((2 * n, 2 * n), complex)
    for i in range(n):
        X[:, 2 * i] = np.concatenate([R[:, i], np.zeros(n)])
        X[:, 2 * i + 1] = np.concatenate([dR[:, i], R[:, i]]) / dlam[i]
        Xi[2 * i] = np.concatenate([np.conj(L[:, i]), np.conj(dL[:, i])])
        Xi[2 * i + 1] = dlam[i] * np.concatenate([np.zeros(n), np.conj(L[:, i])])
    B = matfun.block(A0, dA)
    assert np.abs(Xi @ X - np.eye(2 * n)).max() < 1e-10
    J = np.zeros((2 * n, 2 * n), complex)
    for i in range(n):
        J[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[lam[i], 1], [0, lam[i]]]
    assert np.abs(Xi @ B @ X - J).max() < 1e-9


def test_eigenvector_derivative_identities(setup):
    U, H, dH, b = setup
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, 6)
    for j in range(6):
        res = (H - lam[j] * np.eye(H.shape[0])) @ dR[:, j] - (dlam[j] * R[:, j] - dH @ R[:, j])
        assert np.abs(res).max() < 1e-10
        resl = np.conj(dL[:, j]) @ (H - lam[j] * np.eye(H.shape[0])) - (dlam[j] * np.conj(L[:, j]) - np.conj(L[:, j]) @ dH)
        assert np.abs(resl).max() < 1e-10
        assert abs(np.vdot(L[:, j], dR[:, j])) < 1e-10
        assert abs(np.vdot(dL[:, j], R[:, j])) < 1e-10
    assert np.abs(np.conj(L).T @ R - np.eye(6)).max() < 1e-10


def test_resolvent_split_matches_full_sum(setup):
    """The paper's partial sum + complement resolvent equals the full spectral sum."""
    U, H, dH, b = setup
    l = 4
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, l)
    dl2, dR2, dL2 = deflation.eig_derivs_resolvent(
        lambda v: H @ v, lambda v: H.conj().T @ v, lambda v: dH @ v, lambda v: dH.conj().T @ v,
        H.shape[0], lam, R, L)
    assert np.abs(dl2 - dlam).max() < 1e-11
    assert np.abs(dR2 - dR).max() < 1e-8
    assert np.abs(dL2 - dL).max() < 1e-8


def test_block_projector_invariant(setup):
    """P_{2l} from (R, L, dR, dL) is idempotent and commutes with B."""
    U, H, dH, b = setup
    l = 5
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, l)
    n = H.shape[0]
    B = matfun.block(H, dH)
    P = np.stack([deflation.block_projector_apply(e, R, L, dR, dL)[0] for e in np.eye(2 * n)], axis=1)
    assert np.abs(P @ P - P).max() < 1e-10
    assert np.abs(P @ B - B @ P).max() < 1e-9


def test_projector_derivative_finite_difference(setup):
    """dP = dR L^dag + R dL^dag equals the finite difference of the spectral projector in mu."""
    U, H, dH, b = setup
    l, h = 3, 1e-6
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, l)

    def proj(mu):
        lm, Rm, Lm = deflation.eigpairs_dense(dirac.dense_h(U, DIMS, mu), l)
        return Rm @ np.conj(Lm).T

    fd = (proj(MU + h) - proj(MU - h)) / (2 * h)
    dP = dR @ np.conj(L).T + R @ np.conj(dL).T
    assert np.abs(fd - dP).max() < 1e-6


def test_standard_deflation_exact_and_convergent(setup):
    U, H, dH, b = setup
    h, hd, _, _ = _ops(U)
    ref = matfun.sign_schur(H) @ b
    lam, R, L = deflation.eigpairs_dense(H, 20)
    e_plain = np.linalg.norm(tsl.krylov_sign(h, hd, b, b, 24)[0] - ref)
    e_defl = np.linalg.norm(deflation.deflate_std(h, hd, b, 24, lam, R, L)[0] - ref)
    assert e_defl < e_plain
    y, _ = deflation.deflate_std(h, hd, b, 160, lam, R, L)
    assert np.linalg.norm(y - ref) < 1e-7


def test_generalised_deflation(setup):
    """Eq. 11 for sgn: deflated block method matches the dense derivative and improves on plain."""
    U, H, dH, b = setup
    h, hd, dh, dhd = _ops(U)
    ref = matfun.sign_schur(H) @ b
    dref = matfun.frechet_sign_block(H, dH) @ b
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, 12)
    k = 48
    dy0, _, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, k)
    dy1, y1, _ = deflation.deflate_gen(h, hd, dh, dhd, b, k, lam, R, L, dR, dL)
    assert np.linalg.norm(dy1 - dref) < np.linalg.norm(dy0 - dref)
    dy2, y2, _ = deflation.deflate_gen(h, hd, dh, dhd, b, 240, lam, R, L, dR, dL)
    assert np.linalg.norm(dy2 - dref) / np.linalg.norm(dref) < 1e-6
    assert np.linalg.norm(y2 - ref) < 1e-7
    x = synth.make_source(DIMS, 33).ravel()
    s, _ = deflation.deflate_gen_scalar(h, hd, dh, dhd, b, x, 240, lam, R, L, dR, dL)
    assert abs(s - np.vdot(x, dy2)) < 1e-12


def test_generalised_deflation_link_direction(setup):
    U, H, dH, b = setup
    X = synth.make_su3_direction(DIMS, 34)
    dU = dirac.link_tangent(X, U)
    dHl = dirac.dense_dh_dlink(dU, DIMS, MU)
    h, hd, _, _ = _ops(U)
    dh = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, DIMS, MU))
    dhd = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, DIMS, -MU))
    assert np.abs(dHl.conj().T - dirac.dense_dh_dlink(dU, DIMS, -MU)).max() < 1e-14
    dref = matfun.frechet_sign_block(H, dHl) @ b
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dHl, 12)
    dy, _, _ = deflation.deflate_gen(h, hd, dh, dhd, b, 240, lam, R, L, dR, dL)
    assert np.linalg.norm(dy - dref) / np.linalg.norm(dref) < 1e-6
