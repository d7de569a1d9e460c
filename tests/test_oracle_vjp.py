"""Pins of the oracle's gradient of <x|sgn(H)|b> (no GPU)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import dirac, matfun, vjp

DIMS = (2, 2, 2, 2)
MU = 0.3


@pytest.fixture(scope="module")
def setup():
    U = synth.make_links(DIMS, 0.5, 41)
    x = synth.make_source(DIMS, 42).ravel()
    b = synth.make_source(DIMS, 43).ravel()
    s, dsdmu, F = vjp.dense_vjp(U, DIMS, MU, x, b)
    return U, x, b, s, dsdmu, F


def _s(U, mu, x, b):
    return np.vdot(x, matfun.sign_schur(dirac.dense_h(U, DIMS, mu)) @ b)


def test_dsdmu_finite_difference(setup):
    U, x, b, s, dsdmu, F = setup
    h = 1e-5
    fd = (_s(U, MU + h, x, b) - _s(U, MU - h, x, b)) / (2 * h)
    assert abs(fd - dsdmu) < 1e-8 * max(1, abs(dsdmu))


def test_force_finite_difference(setup):
    U, x, b, s, dsdmu, F = setup
    X = synth.make_su3_direction(DIMS, 44)
    h = 1e-5

    def moved(t):
        E = np.stack([np.stack([expm(t * X[n, v]) for v in range(X.shape[1])]) for n in range(4)])
        return np.einsum("nvab,nvbc->nvac", E, U)

    fd = (_s(moved(h), MU, x, b) - _s(moved(-h), MU, x, b)) / (2 * h)
    an = vjp.directional(F, X)
    assert abs(fd - an) < 1e-8 * max(1, abs(an))


def test_u1_phase_derivative(setup):
    """A U(1) phase on one temporal link: ds/dtheta = i tr F for that link."""
    U, x, b, s, dsdmu, F = setup
    h = 1e-5
    site, nu = 3, 3

    def moved(t):
        Um = U.copy()
        Um[nu, site] = np.exp(1j * t) * Um[nu, site]
        return Um

    fd = (_s(moved(h), MU, x, b) - _s(moved(-h), MU, x, b)) / (2 * h)
    assert abs(fd - 1j * np.trace(F[nu, site])) < 1e-8


def test_u1_derivative_every_link(setup):
    """u1_derivative (i tr F) against central differences of the dense s for
    the U(1) phase of every link of the 2^4 lattice."""
    U, x, b, s, dsdmu, F = setup
    h = 1e-5
    D = vjp.u1_derivative(F)
    for nu in range(4):
        for site in range(U.shape[1]):
            Up, Um = U.copy(), U.copy()
            Up[nu, site] = np.exp(1j * h) * Up[nu, site]
            Um[nu, site] = np.exp(-1j * h) * Um[nu, site]
            fd = (_s(Up, MU, x, b) - _s(Um, MU, x, b)) / (2 * h)
            assert abs(fd - D[nu, site]) < 1e-8, (nu, site)


def test_krylov_vjp_converges_to_dense(setup):
    U, x, b, s, dsdmu, F = setup
    out = [vjp.krylov_vjp(U, DIMS, MU, x, b, k) for k in (40, 160)]
    err_s = [abs(o[0] - s) for o in out]
    err_d = [abs(o[1] - dsdmu) for o in out]
    err_F = [np.abs(o[2] - F).max() for o in out]
    assert err_s[1] < err_s[0] and err_s[1] < 1e-12
    assert err_d[1] < err_d[0] and err_d[1] < 1e-7
    assert err_F[1] < err_F[0] and err_F[1] < 1e-8
