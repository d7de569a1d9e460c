"""Pins of the oracle's Wilson kernel against the mathematics (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, freefield

DIMS = (2, 2, 2, 4)   # N = 384: dense matrices build in well under a second


@pytest.fixture(scope="module")
def links():
    return synth.make_links(DIMS, 0.5, 11)


def test_gamma_algebra():
    G = dirac.GAMMA
    for a in range(4):
        assert np.allclose(G[a], G[a].conj().T)
        for b in range(4):
            assert np.allclose(G[a] @ G[b] + G[b] @ G[a], 2.0 * (a == b) * np.eye(4))
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))


def test_adjoint_is_minus_mu(links):
    """H(mu)^dag = H(-mu): dense check plus the independently coded adjoint."""
    mu = 0.3
    H = dirac.dense_h(links, DIMS, mu)
    Hm = dirac.dense_h(links, DIMS, -mu)
    assert np.abs(H.conj().T - Hm).max() < 1e-14
    v = synth.make_source(DIMS, 3).ravel()
    a = dirac.flat(dirac.apply_hdag(links, v, DIMS, mu))
    assert np.abs(a - H.conj().T @ v).max() < 1e-14


def test_hermitian_at_zero_mu(links):
    H = dirac.dense_h(links, DIMS, 0.0)
    assert np.abs(H - H.conj().T).max() < 1e-14


def test_gauge_covariance(links):
    """H[U^g] = G H[U] G^dag with U^g_nu(x) = g(x) U_nu(x) g(x+nu)^dag."""
    Lx, Ly, Lz, Lt = DIMS
    g = synth.make_gauge_rotation(DIMS, 5)
    g5 = g.reshape(Lt, Lz, Ly, Lx, 3, 3)
    U = links.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    Ug = np.empty_like(U)
    for nu, ax in enumerate((3, 2, 1, 0)):
        gp = np.roll(g5, -1, axis=ax)
        Ug[nu] = np.einsum("...ab,...bc,...dc->...ad", g5, U[nu], np.conj(gp))
    v = synth.make_source(DIMS, 4)
    mu = 0.25
    lhs = dirac.flat(dirac.apply_h(Ug.reshape(4, -1, 3, 3), v, DIMS, mu))
    gv = np.einsum("vab,vsb->vsa", np.conj(g).transpose(0, 2, 1), v)
    rhs = np.einsum("vab,vsb->vsa", g, dirac.flat(dirac.apply_h(links, gv, DIMS, mu)).reshape(-1, 4, 3))
    assert np.abs(lhs - rhs.ravel()).max() < 1e-14


def test_free_spectrum_matches_momentum_formula():
    """Unit links: dense eigenvalues equal the momentum-space 4x4 eigenvalues."""
    V = int(np.prod(DIMS))
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    mu = 0.3
    ev = np.linalg.eigvals(dirac.dense_h(U, DIMS, mu))
    ref = freefield.spectrum(DIMS, mu)
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert np.abs(np.sort_complex(np.round(ev, 10)) - np.sort_complex(np.round(ref, 10))).max() < 1e-8
    del key


def test_free_dirac_closed_form_value():
    """Closed form at one momentum: Dw(p) = m0+4r - r sum cos(pt) + i sum gamma sin(pt)."""
    dims = (2, 2, 2, 2)
    mu, m0 = 0.2, -1.5
    H, dH = freefield.h_of_p(dims, mu, m0)
    # p = (0, 0, 0, pi/2): cos terms 3 + cos(pi/2 - i mu); sin terms only in time
    p4 = np.pi / 2 - 1j * mu
    D = (m0 + 4 - 3 - np.cos(p4)) * np.eye(4) + 1j * np.sin(p4) * dirac.GAMMA[3]
    assert np.allclose(H[0, 0, 0, 0], dirac.GAMMA5 @ D, atol=1e-15)


def test_dmu_finite_difference(links):
    mu, h = 0.3, 1e-5
    v = synth.make_source(DIMS, 6)
    fd = (dirac.flat(dirac.apply_h(links, v, DIMS, mu + h)) - dirac.flat(dirac.apply_h(links, v, DIMS, mu - h))) / (2 * h)
    an = dirac.flat(dirac.apply_dh_dmu(links, v, DIMS, mu))
    assert np.abs(fd - an).max() < 1e-9


def test_dlink_finite_difference(links):
    from scipy.linalg import expm
    mu, h = 0.3, 1e-5
    X = synth.make_su3_direction(DIMS, 8)
    v = synth.make_source(DIMS, 9)

    def moved(t):
        E = np.stack([np.stack([expm(t * X[n, s]) for s in range(X.shape[1])]) for n in range(4)])
        return np.einsum("nvab,nvbc->nvac", E, links)

    fd = (dirac.flat(dirac.apply_h(moved(h), v, DIMS, mu)) - dirac.flat(dirac.apply_h(moved(-h), v, DIMS, mu))) / (2 * h)
    an = dirac.flat(dirac.apply_dh_dlink(dirac.link_tangent(X, links), v, DIMS, mu))
    assert np.abs(fd - an).max() < 1e-9


def test_translation_covariance(links):
    """Shifting links and source by one site in x shifts the result."""
    Lx, Ly, Lz, Lt = DIMS
    mu = 0.3
    v = synth.make_source(DIMS, 10)
    U5 = links.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    v5 = v.reshape(Lt, Lz, Ly, Lx, 4, 3)
    Us = np.roll(U5, 1, axis=4).reshape(4, -1, 3, 3)
    vs = np.roll(v5, 1, axis=3)
    a = np.roll(dirac.apply_h(links, v, DIMS, mu), 1, axis=3)
    b = dirac.apply_h(Us, vs, DIMS, mu)
    assert np.abs(a - b).max() < 1e-14


def test_links_are_su3():
    U = synth.make_links((2, 2, 2, 2), 0.4, 1)
    I = np.einsum("nvab,nvcb->nvac", U, np.conj(U))
    assert np.abs(I - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
