"""Pins of the derivative form of the Sec. 4 error estimate and of the block
sign on a general block source (the second application of that estimate).

  * the exact dense sign of B = [[H, dH], [0, H]] gives eps_B at rounding level
    (sgn(B)^2 = 1 for the block matrix too);
  * the Krylov-Ritz sgn(B) psi for a general psi = (p_t; p_b) converges to the
    dense sgn(B) psi, undeflated and with the generalised deflation of eq. 11;
  * the Krylov eps_B falls with k and stays within a small factor of the true
    error of sgn(B) (0; phi).
"""
import numpy as np
import pytest

import synth
from oracle import deflation, dirac, estimator, matfun, tsl

DIMS, MU = (4, 2, 2, 4), 0.3


@pytest.fixture(scope="module")
def setup():
    U = synth.make_links(DIMS, 1.0, 301)
    H = dirac.dense_h(U, DIMS, MU)
    dH = dirac.dense_dh_dmu(U, DIMS, MU)
    SB = matfun.sign_schur(matfun.block(H, dH))
    h = lambda v: dirac.flat(dirac.apply_h(U, v, DIMS, MU))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, DIMS, MU))
    dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, MU))
    dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, DIMS, -MU))
    return U, H, dH, SB, (h, hd, dh, dhd)


def test_exact_block_sign_gives_rounding_level_eps(setup):
    U, H, dH, SB, _ = setup
    phi = synth.make_source(DIMS, 5).ravel()
    assert estimator.eps_block(lambda v: SB @ v, phi) < 1e-12


def test_general_block_source_converges_to_dense(setup):
    U, H, dH, SB, ops = setup
    n = H.shape[0]
    psi = np.concatenate([synth.make_source(DIMS, 6).ravel(), synth.make_source(DIMS, 7).ravel()])
    ref = SB @ psi
    errs = []
    for k in (64, 400, 800):   # 2N = 1536; measured 0.11, 9.5e-5, 3.9e-12
        y, _ = tsl.krylov_block_sign(*ops, psi, k)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10, errs
    # with the generalised deflation (eq. 11) of the 10 pairs closest to zero
    # (this rough field has a small gap): measured 4.9e-8 at k = 400
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, 10)
    yd, _ = deflation.deflate_gen_block(*ops, psi, 400, lam, R, L, dR, dL)
    ed = np.linalg.norm(yd - ref) / np.linalg.norm(ref)
    assert ed < 1e-2 * errs[1], (ed, errs)
    # a top half of zero reduces to the derivative form of eq. 7
    b = psi[n:]
    y0, _ = deflation.deflate_gen_block(*ops, np.concatenate([np.zeros(n), b]), 64, lam, R, L, dR, dL)
    d1, y1, _ = deflation.deflate_gen(*ops, b, 64, lam, R, L, dR, dL)
    assert np.allclose(y0, np.concatenate([d1, y1]), rtol=0, atol=1e-13)


def test_krylov_eps_block_decreases_and_tracks_the_error(setup):
    U, H, dH, SB, ops = setup
    phi = synth.make_source(DIMS, 8).ravel()
    psi = np.concatenate([np.zeros_like(phi), phi])
    ref = SB @ psi
    prev = None
    for k in (48, 96, 192):   # measured eps / error: 0.72, 0.63, 0.87
        app = lambda v: tsl.krylov_block_sign(*ops, v, k)[0]
        eps = estimator.eps_block(app, phi)
        err = np.linalg.norm(app(psi) - ref) / np.linalg.norm(ref)
        assert 0.2 * err < eps < 5 * err, (k, eps, err)
        if prev is not None:
            assert eps < prev
        prev = eps
