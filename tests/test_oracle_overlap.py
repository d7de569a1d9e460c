"""Pins of the oracle's overlap operator (eq. 1), no GPU."""
import numpy as np

import synth
from oracle import overlap

DIMS = (2, 2, 2, 2)


def test_ginsparg_wilson_relation():
    U = synth.make_links(DIMS, 0.5, 61)
    for mu in (0.0, 0.3):
        D = overlap.dense_overlap(U, DIMS, mu)
        G5 = overlap.gamma5_field(D.shape[0])
        assert np.abs(G5 @ D + D @ G5 - D @ G5 @ D).max() < 1e-10


def test_circle_and_gamma5_hermiticity_at_zero_mu():
    U = synth.make_links(DIMS, 0.5, 62)
    D = overlap.dense_overlap(U, DIMS, 0.0)
    G5 = overlap.gamma5_field(D.shape[0])
    lam = np.linalg.eigvals(D)
    assert np.abs(np.abs(lam - 1.0) - 1.0).max() < 1e-10
    assert np.abs(D.conj().T - G5 @ D @ G5).max() < 1e-10


def test_krylov_overlap_converges_to_dense():
    U = synth.make_links(DIMS, 0.5, 63)
    b = synth.make_source(DIMS, 64).ravel()
    D = overlap.dense_overlap(U, DIMS, 0.3)
    errs = [np.linalg.norm(overlap.krylov_overlap(U, DIMS, 0.3, b, k) - D @ b) for k in (40, 120, 180)]
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-6


def test_krylov_overlap_derivative_against_dense():
    """d/dmu D_ov b = gamma5 L_sgn(H, dH/dmu) b: the oracle's Krylov form (block
    Lanczos of eq. 6-7, with its own adjoint of dH/dmu) converges to gamma5 times
    the dense Frechet derivative (top-right block of sgn([[H, dH], [0, H]]),
    pinned in test_oracle_matfun).  Measured: 3.9e-3 at k = 100, 9.7e-7 at 200,
    1.4e-10 at 300 (2N = 384)."""
    from oracle import dirac, matfun
    mu = 0.3
    U = synth.make_links(DIMS, 0.5, 61)
    b = synth.make_source(DIMS, 62).ravel()
    H = dirac.dense_h(U, DIMS, mu)
    dH = dirac.dense_dh_dmu(U, DIMS, mu)
    g5 = np.tile(np.repeat(np.diag(dirac.GAMMA5).real, 3), b.size // 12)
    ref = g5 * (matfun.frechet_sign_block(H, dH) @ b)
    errs = [np.linalg.norm(overlap.krylov_overlap_deriv(U, DIMS, mu, b, k) - ref) / np.linalg.norm(ref)
            for k in (100, 200, 300)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-9, errs
