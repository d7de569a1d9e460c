"""Deflation of the sign function and of its derivative -- oracle (test infrastructure only).

Sec. 3, eq. 8 (standard deflation): with right/left eigenvectors R_i, L_i of A
(L_i^dag R_j = delta_ij) for the m eigenvalues closest to zero,

    sgn(A) x = sum_{i<=m} sgn(lambda_i) R_i <L_i|x>  +  sgn(A) P x,
    P = 1 - sum_{i<=m} R_i L_i^dag,

the first part exact, the second by the Krylov-Ritz method.

Sec. 3, eq. 9-11 (generalised deflation of the block matrix B = [[A, dA], [0, A]]):
B has 2x2 Jordan blocks; eq. 10 writes its Jordan basis with columns
X_{2i-1} = (R_i; 0), X_{2i} = (dR_i; R_i)/dlambda_i and rows
Xbar_{2i-1} = (L_i^dag, dL_i^dag), Xbar_{2i} = dlambda_i (0, L_i^dag).
For the sign function the mixing terms of eq. 11 vanish, so with the l
eigenvalues closest to zero

    sgn(B) psi = sgn(B) Pbar_{2l} psi + sum_{i=1}^{2l} sgn(lambda_{ceil(i/2)}) X_i <Xbar_i|psi>.

Readings (recorded in the design notes):
  * the eigenvalue attached to X_i in the last sum is that of Jordan block
    ceil(i/2);
  * in X_{2i} Xbar_{2i} the factors 1/dlambda_i and dlambda_i cancel, so the
    code multiplies (dR_i; R_i) by <(0, L_i^dag)|psi> and never divides;
  * the left start of the deflated block Lanczos run uses the same rule as
    without deflation, applied to the projected source;
  * eigenvector derivatives (the garbled end of Sec. 3) are read as the
    standard first-order perturbation formulas with the gauge
    L_j^dag dR_j = 0 and dL_j^dag R_j = 0:
        dR_j   = sum_{i != j} R_i (L_i^dag dA R_j)/(lambda_j - lambda_i)
        dL_j^dag = sum_{i != j} (L_j^dag dA R_i) L_i^dag/(lambda_j - lambda_i)
    where the sum over i > l is the complement resolvent
    (lambda_j - A)^{-1} Pbar_l, as the paper indicates.

Pinned by (tests/test_oracle_deflation.py): the block projector built from
(R, L, dR, dL) is idempotent and commutes with B; the residual identity
(A - lambda_j) dR_j = (dlambda_j - dA) R_j and the gauge conditions; finite
differences of the spectral projector; deflated and undeflated Krylov-Ritz
results agree with the dense sign and its dense derivative.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import matfun, tsl


def eigpairs_dense(A, m):
    """m eigenpairs of smallest |lambda|: lam (m), R (n x m), L (n x m) with L^dag R = I."""
    lam, S = np.linalg.eig(A)
    Si = np.linalg.inv(S)
    order = np.argsort(np.abs(lam), kind="stable")[:m]
    return lam[order], S[:, order], np.conj(Si[order, :]).T


def eig_derivs_dense(A, dA, m):
    """Eigenpairs and their t-derivatives along dA from a full dense eigendecomposition.

    Returns lam, R, L, dlam, dR, dL (first m by |lambda|), with the gauge
    L_j^dag dR_j = 0 = dL_j^dag R_j.
    """
    lam_all, S = np.linalg.eig(A)
    Si = np.linalg.inv(S)
    order = np.argsort(np.abs(lam_all), kind="stable")
    lam_all, S, Si = lam_all[order], S[:, order], Si[order, :]
    G = Si @ dA @ S                     # G_ij = L_i^dag dA R_j
    n = A.shape[0]
    lam = lam_all[:m]
    dlam = np.diag(G)[:m].copy()
    dR = np.zeros((n, m), dtype=np.complex128)
    dLh = np.zeros((m, n), dtype=np.complex128)   # rows dL_j^dag
    for j in range(m):
        den = lam_all[j] - lam_all
        den[j] = 1.0
        cj = G[:, j] / den
        cj[j] = 0.0
        dR[:, j] = S @ cj
        rj = G[j, :] / den
        rj[j] = 0.0
        dLh[j, :] = rj @ Si
    return lam, S[:, :m], np.conj(Si[:m, :]).T, dlam, dR, np.conj(dLh).T


def eig_derivs_resolvent(apply_a, apply_a_h, apply_da, apply_da_h, n, lam, R, L, tol=1e-12):
    """Eigenvector derivatives by the paper's split: a partial sum over the l
    deflated pairs plus the complement resolvent (lambda_j - A)^{-1} Pbar.

    ``apply_*`` act on flat vectors (A, A^dag, dA, dA^dag).  The complement
    solves use GMRES on (lambda_j - A) Pbar + P, which is invertible and equals
    (lambda_j - A) on range(Pbar); the left ones use its adjoint.
    Returns dlam, dR, dL (dL as columns, i.e. dL_j^dag is a row of dL^dag).
    """
    l = lam.size
    Lh = np.conj(L).T
    Rh = np.conj(R).T
    dAR = np.stack([apply_da(R[:, j]) for j in range(l)], axis=1)
    dAhL = np.stack([apply_da_h(L[:, j]) for j in range(l)], axis=1)
    G = Lh @ dAR                                    # G_ij = L_i^dag dA R_j
    dR = np.zeros((n, l), dtype=np.complex128)
    dL = np.zeros((n, l), dtype=np.complex128)
    dlam = np.diag(G).copy()

    def pbar(v):
        return v - R @ (Lh @ v)

    def pbar_h(v):
        return v - L @ (Rh @ v)

    def solve(matvec, rhs):
        op = spla.LinearOperator((n, n), dtype=np.complex128, matvec=matvec)
        x, info = spla.gmres(op, rhs, rtol=tol, atol=0.0, restart=300, maxiter=300)
        if info != 0:
            raise RuntimeError("complement resolvent solve did not converge")
        return x

    for j in range(l):
        lj = lam[j]
        x = solve(lambda v: lj * pbar(v) - apply_a(pbar(v)) + R @ (Lh @ v), pbar(dAR[:, j]))
        xl = solve(lambda v: np.conj(lj) * pbar_h(v) - apply_a_h(pbar_h(v)) + L @ (Rh @ v),
                   pbar_h(dAhL[:, j]))
        part_r = np.zeros(n, dtype=np.complex128)
        part_l = np.zeros(n, dtype=np.complex128)
        for i in range(l):
            if i != j:
                part_r += R[:, i] * (G[i, j] / (lj - lam[i]))
                part_l += L[:, i] * np.conj(G[j, i] / (lj - lam[i]))
        dR[:, j] = part_r + pbar(x)
        dL[:, j] = part_l + pbar_h(xl)
    return dlam, dR, dL


def deflate_std(op, op_h, b, k, lam, R, L, sign=matfun.sign_schur, tau=1e-14):
    """Eq. 8: exact part on span(R) plus Krylov-Ritz sign on the projected source."""
    c = np.conj(L).T @ b
    bp = b - R @ c
    y, info = tsl.krylov_sign(op, op_h, bp, bp, k, sign, tau)
    return y + R @ (matfun.sgn_scalar(lam) * c), info


def block_projector_apply(psi, R, L, dR, dL):
    """P_{2l} psi with the block projector [[P, dP], [0, P]] of eq. 10-11."""
    n = R.shape[0]
    pt, pb = psi[:n], psi[n:]
    Lh, dLh = np.conj(L).T, np.conj(dL).T
    c_t = Lh @ pt + dLh @ pb       # <Xbar_{2i-1}|psi>
    c_b = Lh @ pb                  # <Xbar_{2i}|psi> / dlambda_i
    top = R @ c_t + dR @ c_b
    bot = R @ c_b
    return np.concatenate([top, bot]), c_t, c_b


def deflate_gen(h, h_dag, dh, dh_dag, b, k, lam, R, L, dR, dL,
                sign=matfun.sign_schur, rule="sum", tau=1e-14):
    """Eq. 11 for the sign: (d sgn(A) b, sgn(A) b) with l deflated Jordan blocks."""
    n = b.size
    psi = np.concatenate([np.zeros(n, dtype=np.complex128), b.ravel()])
    proj, c_t, c_b = block_projector_apply(psi, R, L, dR, dL)
    psi_p = psi - proj
    op, op_h = tsl.block_ops(h, h_dag, dh, dh_dag, n)
    phi = tsl.block_left_start(psi_p, n, rule)
    y, info = tsl.krylov_sign(op, op_h, psi_p, phi, k, sign, tau)
    s = matfun.sgn_scalar(lam)
    exact_top = R @ (s * c_t) + dR @ (s * c_b)
    exact_bot = R @ (s * c_b)
    return y[:n] + exact_top, y[n:] + exact_bot, info


def deflate_gen_block(h, h_dag, dh, dh_dag, psi, k, lam, R, L, dR, dL,
                      sign=matfun.sign_schur, rule="sum", tau=1e-14):
    """Eq. 11 for a general block source psi = (p_t; p_b): sgn(B) psi as one
    2n vector, l deflated Jordan blocks."""
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    n = psi.size // 2
    proj, c_t, c_b = block_projector_apply(psi, R, L, dR, dL)
    psi_p = psi - proj
    op, op_h = tsl.block_ops(h, h_dag, dh, dh_dag, n)
    phi = tsl.block_left_start(psi_p, n, rule)
    y, info = tsl.krylov_sign(op, op_h, psi_p, phi, k, sign, tau)
    s = matfun.sgn_scalar(lam)
    exact = np.concatenate([R @ (s * c_t) + dR @ (s * c_b), R @ (s * c_b)])
    return y + exact, info


def deflate_gen_scalar(h, h_dag, dh, dh_dag, b, x, k, lam, R, L, dR, dL,
                       sign=matfun.sign_schur, rule="sum", tau=1e-14):
    """<x| d sgn(A) b> in the storage-free scalar mode, with generalised deflation."""
    n = b.size
    psi = np.concatenate([np.zeros(n, dtype=np.complex128), b.ravel()])
    proj, c_t, c_b = block_projector_apply(psi, R, L, dR, dL)
    psi_p = psi - proj
    op, op_h = tsl.block_ops(h, h_dag, dh, dh_dag, n)
    phi = tsl.block_left_start(psi_p, n, rule)
    xx = np.concatenate([x.ravel(), np.zeros(n, dtype=np.complex128)])
    val, info = tsl.krylov_sign_scalar(op, op_h, psi_p, phi, k, xx, sign, tau)
    s = matfun.sgn_scalar(lam)
    exact = np.vdot(x, R @ (s * c_t) + dR @ (s * c_b))
    return val + exact, info
