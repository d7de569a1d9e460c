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


def test_deflated_krylov_vjp_against_dense():
    """The deflated gradient (12 eigenpairs of the rough 4x2x2x4 field, dense
    eigen-data) converges to the dense gradient, faster than the undeflated
    form (measured at k = 256: ds/dmu 1.3e-6 against 4.3e-4, force 2.4e-6
    against 4.0e-4; at k = 600 all below 1e-12), and with no pairs it is the
    undeflated form."""
    from oracle import deflation
    dims = (4, 2, 2, 4)
    U = synth.make_links(dims, 1.0, 301)
    x = synth.make_source(dims, 42).ravel()
    b = synth.make_source(dims, 43).ravel()
    s, dsdmu, F = vjp.dense_vjp(U, dims, MU, x, b)
    H = dirac.dense_h(U, dims, MU)
    lam, R, L = deflation.eigpairs_dense(H, 12)
    err = lambda o: (abs(o[0] - s) / abs(s), abs(o[1] - dsdmu) / abs(dsdmu), np.abs(o[2] - F).max() / np.abs(F).max())
    e_u = err(vjp.krylov_vjp(U, dims, MU, x, b, 256))
    e_d = err(vjp.krylov_vjp_deflated(U, dims, MU, x, b, 256, lam, R, L))
    assert all(d < 0.05 * u for d, u in zip(e_d, e_u)), (e_d, e_u)
    e_600 = err(vjp.krylov_vjp_deflated(U, dims, MU, x, b, 600, lam, R, L))
    assert max(e_600) < 1e-10, e_600
    o0 = vjp.krylov_vjp(U, dims, MU, x, b, 48)
    o1 = vjp.krylov_vjp_deflated(U, dims, MU, x, b, 48, lam[:0], R[:, :0], L[:, :0])
    assert abs(o1[0] - o0[0]) < 1e-14 and abs(o1[1] - o0[1]) < 1e-14 and np.abs(o1[2] - o0[2]).max() < 1e-14
