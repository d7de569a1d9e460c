"""The overlap operator of eq. 1 -- oracle (test infrastructure only).

D_ov = (1/a)(1 + gamma5 sgn(H(mu))) with H(mu) = gamma5 Dw(mu) (Sec. 1, eq. 1);
here a = 1.  Its derivative along t is gamma5 d/dt sgn(H) (the identity does
not depend on t).

Pinned by (tests/test_oracle_overlap.py): the Ginsparg-Wilson relation
gamma5 D + D gamma5 = D gamma5 D (which holds for any S with S^2 = 1), the
eigenvalues of D at mu = 0 on the circle |z - 1| = 1, gamma5-hermiticity
D^dag = gamma5 D gamma5 at mu = 0, and the Krylov derivative converging to
gamma5 times the dense Frechet derivative of the sign.
"""
from __future__ import annotations

import numpy as np

from . import dirac, matfun, tsl


def gamma5_field(n):
    """gamma5 on a flat field of n = 12 V complex (spin-major within a site)."""
    g = np.tile(np.repeat(np.diag(dirac.GAMMA5).real, 3), n // 12)
    return np.diag(g.astype(np.complex128))


def dense_overlap(U, dims, mu, m0=-1.5):
    """D_ov as a dense matrix, with the Schur-based sign."""
    H = dirac.dense_h(U, dims, mu, m0)
    G5 = gamma5_field(H.shape[0])
    return np.eye(H.shape[0]) + G5 @ matfun.sign_schur(H)


def krylov_overlap(U, dims, mu, b, k, m0=-1.5):
    """D_ov b with the k-step two-sided Lanczos sign (start b, left start b)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0))
    y, _ = tsl.krylov_sign(h, hd, b, b, k)
    g5 = np.tile(np.repeat(np.diag(dirac.GAMMA5).real, 3), b.size // 12)
    return b + g5 * y


def krylov_overlap_deriv(U, dims, mu, b, k, m0=-1.5):
    """d/dmu D_ov b = gamma5 d/dmu sgn(H) b with the block-matrix Lanczos (eq. 6-7)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0))
    dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, dims, mu))
    dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, dims, -mu))
    d, _, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b, k)
    g5 = np.tile(np.repeat(np.diag(dirac.GAMMA5).real, 3), b.size // 12)
    return g5 * d
