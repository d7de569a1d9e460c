"""Error estimate of Sec. 4 -- oracle (test infrastructure only).

Sec. 4 estimates the relative error of a sign-function evaluation from
sgn(A)^2 = 1:  eps_A = |sgn(A)^2 psi - psi| / (2 |psi|), the factor two
because the approximation is applied twice; for the derivative the same is
done with the block matrix B and the source (0, phi)^T.

Pinned by (tests/test_oracle_tsl.py): eps_A is at rounding level for the dense
sign and decreases with the Krylov size for the Krylov-Ritz approximation.
"""
from __future__ import annotations

import numpy as np


def eps_sign(apply_sign, psi):
    """eps_A for a callable that applies (an approximation of) sgn(A)."""
    psi = np.asarray(psi).ravel()
    return np.linalg.norm(apply_sign(apply_sign(psi)) - psi) / (2 * np.linalg.norm(psi))
