"""Error estimate of Sec. 4 -- oracle (test infrastructure only).

Sec. 4 estimates the relative error of a sign-function evaluation from
sgn(A)^2 = 1:  eps_A = |sgn(A)^2 psi - psi| / (2 |psi|), the factor two
because the approximation is applied twice; for the derivative the same is
done with the block matrix B of eq. 6 and the sparse source (0, phi)^T, the
second application acting on the full block vector sgn(B) (0, phi)^T.

Pinned by (tests/test_oracle_tsl.py, tests/test_oracle_estimator.py): eps is
at rounding level for the exact dense sign (of A, and of B through the block
identity of eq. 6), it decreases with the Krylov size for the Krylov-Ritz
approximation, and it tracks the true error of the approximation.
"""
from __future__ import annotations

import numpy as np


def eps_sign(apply_sign, psi):
    """eps_A for a callable that applies (an approximation of) sgn(A)."""
    psi = np.asarray(psi).ravel()
    return np.linalg.norm(apply_sign(apply_sign(psi)) - psi) / (2 * np.linalg.norm(psi))


def eps_block(apply_block_sign, phi):
    """eps_B for the derivative: psi = (0; phi), a callable applying (an
    approximation of) sgn(B) to 2n vectors."""
    phi = np.asarray(phi, dtype=np.complex128).ravel()
    psi = np.concatenate([np.zeros_like(phi), phi])
    return eps_sign(apply_block_sign, psi)
