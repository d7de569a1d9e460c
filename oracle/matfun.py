"""Matrix sign function and its derivative on dense matrices -- oracle (test infrastructure only).

Sec. 2, eq. 2-5: f(A) = X f(J) X^{-1}; for diagonalisable A the spectral form
f(A) = X diag(f(lambda_i)) X^{-1}.  For the sign function the paper notes the
discontinuity on the imaginary axis (Sec. 3), i.e. sgn(z) = sgn(Re z); a value
with Re z = 0 is taken as +1 here (a reading; such spectra never occur in the
workloads).

Three independent dense evaluations are provided:
  * ``sign_eig``   -- the spectral form of Sec. 2;
  * ``sign_schur`` -- complex Schur form ordered so that the right-half-plane
    eigenvalues come first, sgn(R) = [[I, Y], [0, -I]] with Y from the
    Sylvester equation R11 Y - Y R22 = 2 R12 (Higham, Functions of Matrices,
    the Schur method for the sign); unlike the spectral form it stays accurate
    when eigenvalues within one half-plane cluster or A is not diagonalisable
    (the block matrix of eq. 6 never is, Sec. 3);
  * ``sign_newton`` -- Newton's iteration X <- (X + X^{-1})/2 with determinant
    scaling (Higham, Functions of Matrices, the scaled Newton iteration).

The derivative (eq. 6, Mathias' theorem): f([[A, E], [0, A]]) has the
directional (Frechet) derivative L_f(A, E) in its top-right block.  An
independent check is the divided-difference formula in an eigenbasis,
``frechet_sign_dd``: with A = S diag(l) S^{-1}, L = S (F o (S^{-1} E S)) S^{-1},
F_ij = (s_i - s_j)/(l_i - l_j) (zero when s_i = s_j).

Pinned by (tests/test_oracle_matfun.py): sgn^2 = 1, agreement of the three
methods on well-conditioned matrices, the scalar case, commutation with A,
the block identity against divided differences and central finite differences.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def sgn_scalar(z):
    """sgn(z) = sgn(Re z), with +1 on the imaginary axis."""
    z = np.asarray(z)
    return np.where(np.real(z) >= 0, 1.0, -1.0)


def sign_eig(A):
    """Spectral form S diag(sgn(Re l)) S^{-1} (eq. 4 for diagonal J)."""
    lam, S = np.linalg.eig(A)
    return (S * sgn_scalar(lam)) @ np.linalg.inv(S)


def sign_schur(A):
    """Schur method: Q [[I, Y], [0, -I]] Q^H with R11 Y - Y R22 = 2 R12."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    R, Q, p = sla.schur(A, output="complex", sort=lambda z: np.real(z) >= 0)
    S = np.zeros((n, n), dtype=np.complex128)
    S[:p, :p] = np.eye(p)
    S[p:, p:] = -np.eye(n - p)
    if 0 < p < n:
        # solve_sylvester solves a X + X b = q
        S[:p, p:] = sla.solve_sylvester(R[:p, :p], -R[p:, p:], 2.0 * R[:p, p:])
    return Q @ S @ Q.conj().T


def sign_newton(A, tol=1e-14, maxit=100):
    """Scaled Newton iteration for the matrix sign."""
    X = np.asarray(A, dtype=np.complex128).copy()
    n = X.shape[0]
    for it in range(maxit):
        Xi = np.linalg.inv(X)
        if it < 10:
            # determinantal scaling |det X|^{-1/n}
            _, logdet = np.linalg.slogdet(X)
            mu = np.exp(-logdet / n)
        else:
            mu = 1.0
        Xn = 0.5 * (mu * X + Xi / mu)
        if np.linalg.norm(Xn - X, 1) <= tol * np.linalg.norm(Xn, 1) and it >= 10:
            return Xn
        X = Xn
    return X


def block(A, E):
    """The 2n x 2n block matrix [[A, E], [0, A]] of eq. 6."""
    n = A.shape[0]
    Z = np.zeros((n, n), dtype=np.complex128)
    return np.block([[A, E], [Z, A]])


def frechet_sign_block(A, E, method=sign_schur):
    """Top-right block of sgn([[A, E], [0, A]]) (eq. 6)."""
    n = A.shape[0]
    return method(block(A, E))[:n, n:]


def frechet_sign_dd(A, E):
    """Divided-difference formula for the derivative of sgn at A along E."""
    lam, S = np.linalg.eig(A)
    Si = np.linalg.inv(S)
    s = sgn_scalar(lam)
    ds = s[:, None] - s[None, :]
    dl = lam[:, None] - lam[None, :]
    F = np.zeros_like(dl)
    mask = ds != 0
    F[mask] = ds[mask] / dl[mask]
    return S @ (F * (Si @ E @ S)) @ Si
