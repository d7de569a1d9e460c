"""Two-sided Lanczos (TSL) Krylov-Ritz approximation -- oracle (test infrastructure only).

Sec. 2 (end): the sign function of the non-Hermitian kernel is applied to a
vector with the two-sided Lanczos method of the cited references, and eq. 7
says any such approximation can be applied to the block matrix
B = [[A, dA], [0, A]] with source (0; x) to obtain (d_t f(A) x ; f(A) x).

The paper cites but does not print the TSL algorithm.  This module writes out
the textbook Lanczos biorthogonalisation (Saad, Iterative Methods for Sparse
Linear Systems, Sec. 7.1) in complex form, with the Krylov-Ritz approximation
f(A) psi ~ |psi| V_k f(T_k) e_1:

  v_1 = psi/|psi|,  w_1 = phi / conj(phi^dag v_1)          (w_1^dag v_1 = 1)
  for j = 1..k:
      u = A v_j,  z = A^dag w_j,  alpha_j = w_j^dag u
      (stop after alpha_k)
      vh = u - alpha_j v_j - beta_j v_{j-1}
      wh = z - conj(alpha_j) w_j - conj(delta_j) w_{j-1}
      omega = wh^dag vh ;  breakdown if |omega| <= tau |wh| |vh|
      delta_{j+1} = sqrt|omega|,  beta_{j+1} = omega / delta_{j+1}
      v_{j+1} = vh / delta_{j+1},  w_{j+1} = wh / conj(beta_{j+1})
  T_k = tridiag(sub = delta_2..delta_k, diag = alpha_1..alpha_k, super = beta_2..beta_k)

Readings of points the paper leaves open (each recorded in the design notes):
  * the normalisation split delta = sqrt|omega| (a convention);
  * breakdown tolerance tau = 1e-14, no look-ahead;
  * sgn(T_k) e_1 by the Schur method (matfun.sign_schur) -- robust when the
    Ritz values pair up, as they do for the non-diagonalisable block matrix --
    or by the paper's nested two-sided Lanczos (``NestedSign``, Sec. 4);
  * left start vector: phi = psi for the kernel itself; for the block system
    (source (p_t; p_b)) phi = (p_t + p_b; p_b).  phi = psi cannot work there:
    B^dag (0; v) = (0; A^dag v), so every left vector would keep a zero top
    half and the top half of the result (the derivative) would be unchecked.

The scalar mode returns <x|y> = |psi| sum_j c_j <x|v_j> without forming y,
which is the storage-free form of the derivative of <x|sgn(H)|b>.

Pinned by (tests/test_oracle_tsl.py): at k = n the Krylov-Ritz result equals
the dense sign; the error against the dense result falls as k grows; at mu = 0
with phi = psi the recurrence is Hermitian Lanczos (T real symmetric); the
biorthogonality W^dag V = 1 and the three-term relation A V = V T + r e_k^T.
"""
from __future__ import annotations

import numpy as np

from . import matfun


class Breakdown(RuntimeError):
    def __init__(self, step, margin):
        super().__init__(f"two-sided Lanczos breakdown at step {step} (|omega|/(|w||v|) = {margin:.3e})")
        self.step = step
        self.margin = margin


def lanczos(op, op_h, psi, phi, k, tau=1e-14, keep_basis=True, proj=None):
    """Run k steps of two-sided Lanczos.

    op, op_h : callables applying A and A^dag to a flat complex vector.
    Returns dict with alpha (k), beta (k+1, beta[j] = beta_{j}, beta[0]=beta[1]=unused),
    delta (k+1), T (k x k), V (n x k) and W (n x k) if keep_basis, norm = |psi|,
    and ``proj`` (k) = <proj|v_j> when a projection vector is given.
    """
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    phi = np.asarray(phi, dtype=np.complex128).ravel()
    n = psi.size
    nrm = np.linalg.norm(psi)
    v = psi / nrm
    w = phi / np.conj(np.vdot(phi, v))
    v_prev = np.zeros(n, dtype=np.complex128)
    w_prev = np.zeros(n, dtype=np.complex128)
    alpha = np.zeros(k, dtype=np.complex128)
    beta = np.zeros(k + 1, dtype=np.complex128)
    delta = np.zeros(k + 1, dtype=np.complex128)
    V = np.empty((n, k), dtype=np.complex128) if keep_basis else None
    W = np.empty((n, k), dtype=np.complex128) if keep_basis else None
    p = np.zeros(k, dtype=np.complex128)
    min_margin = np.inf
    for j in range(k):
        if keep_basis:
            V[:, j] = v
            W[:, j] = w
        if proj is not None:
            p[j] = np.vdot(proj, v)
        u = op(v)
        z = op_h(w)
        alpha[j] = np.vdot(w, u)
        if j == k - 1:
            break
        vh = u - alpha[j] * v - beta[j] * v_prev
        wh = z - np.conj(alpha[j]) * w - np.conj(delta[j]) * w_prev
        omega = np.vdot(wh, vh)
        margin = abs(omega) / (np.linalg.norm(wh) * np.linalg.norm(vh))
        min_margin = min(min_margin, margin)
        if margin <= tau:
            raise Breakdown(j + 1, margin)
        delta[j + 1] = np.sqrt(abs(omega))
        beta[j + 1] = omega / delta[j + 1]
        v_prev, w_prev = v, w
        v = vh / delta[j + 1]
        w = wh / np.conj(beta[j + 1])
    T = np.diag(alpha) + np.diag(beta[1:k], 1) + np.diag(delta[1:k], -1)
    return dict(alpha=alpha, beta=beta, delta=delta, T=T, V=V, W=W, norm=nrm,
                proj=p if proj is not None else None, min_margin=min_margin)


def ritz_coeffs(T, sign=matfun.sign_schur):
    """c = sgn(T_k) e_1.  ``sign`` maps a square matrix to its sign; a
    ``NestedSign`` instance returns the first column directly."""
    if isinstance(sign, NestedSign):
        return sign(T)
    return sign(T)[:, 0]


class NestedSign:
    """sgn(T) e_1 by one level of nesting (Sec. 4: the paper's outer Ritz
    matrix is signed by a nested two-sided Lanczos run, inner Krylov size 100;
    the construction follows the cited nested Krylov-Ritz method).

    The inner run cannot use T itself: its Krylov space from e_1 is spanned by
    e_1 .. e_kp and would only reproduce the outer run truncated at kp steps.
    It uses Tt = (T + T^{-1}) / 2, which has the same sign function as T
    (Re(z + 1/z) = Re z (1 + 1/|z|^2)), with right and left start e_1:

        sgn(T) e_1 ~ V' sgn(T') e_1,   T' the kp x kp inner Ritz matrix,

    and sgn(T') by the dense ``inner`` method.  Tt is formed densely here; at
    kp = k the inner space is all of C^k and the result is exact.

    Pinned by (tests/test_oracle_nested.py): sgn(Tt) = sgn(T) on dense
    matrices, exactness at kp = k against the Schur sign, and convergence in kp
    towards sgn(T) e_1 for the Ritz matrix of a lattice operator.
    """

    def __init__(self, kp, inner=matfun.sign_schur, tau=1e-14):
        self.kp = int(kp)
        self.inner = inner
        self.tau = tau

    def __call__(self, T):
        T = np.asarray(T, dtype=np.complex128)
        k = T.shape[0]
        Tt = 0.5 * (T + np.linalg.inv(T))
        Tth = Tt.conj().T
        e1 = np.zeros(k, dtype=np.complex128)
        e1[0] = 1.0
        L = lanczos(lambda v: Tt @ v, lambda w: Tth @ w, e1, e1, min(self.kp, k), self.tau)
        return L["norm"] * (L["V"] @ self.inner(L["T"])[:, 0])


def krylov_sign(op, op_h, psi, phi, k, sign=matfun.sign_schur, tau=1e-14):
    """sgn(A) psi ~ |psi| V_k sgn(T_k) e_1."""
    L = lanczos(op, op_h, psi, phi, k, tau)
    c = ritz_coeffs(L["T"], sign)
    return L["norm"] * (L["V"] @ c), L


def krylov_sign_scalar(op, op_h, psi, phi, k, x, sign=matfun.sign_schur, tau=1e-14):
    """<x| sgn(A) psi> ~ |psi| sum_j c_j <x|v_j>, without storing the basis."""
    L = lanczos(op, op_h, psi, phi, k, tau, keep_basis=False, proj=x)
    c = ritz_coeffs(L["T"], sign)
    return L["norm"] * np.dot(L["proj"], c), L


# --- block system of eq. 6-7 -------------------------------------------------

def block_ops(h, h_dag, dh, dh_dag, n):
    """Apply B = [[H, dH], [0, H]] and B^dag = [[H^dag, 0], [dH^dag, H^dag]] to 2n vectors."""
    def op(v):
        vt, vb = v[:n], v[n:]
        return np.concatenate([h(vt) + dh(vb), h(vb)])

    def op_h(w):
        wt, wb = w[:n], w[n:]
        return np.concatenate([h_dag(wt), dh_dag(wt) + h_dag(wb)])

    return op, op_h


def block_left_start(psi, n, rule="sum"):
    """Left start vector for the block system: 'sum' -> (p_t + p_b; p_b), 'same' -> psi."""
    if rule == "same":
        return psi.copy()
    return np.concatenate([psi[:n] + psi[n:], psi[n:]])


def krylov_block_sign(h, h_dag, dh, dh_dag, psi, k, sign=matfun.sign_schur, rule="sum", tau=1e-14):
    """sgn(B) psi for a general block vector psi = (p_t; p_b) of length 2n
    (eq. 7 with a full source), left start by ``rule``; returns (y, lanczos info)."""
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    n = psi.size // 2
    op, op_h = block_ops(h, h_dag, dh, dh_dag, n)
    return krylov_sign(op, op_h, psi, block_left_start(psi, n, rule), k, sign, tau)


def krylov_sign_deriv(h, h_dag, dh, dh_dag, b, k, sign=matfun.sign_schur, rule="sum", tau=1e-14):
    """(d sgn(A) b, sgn(A) b) from the Krylov-Ritz approximation of sgn(B) (0; b) (eq. 7)."""
    n = b.size
    op, op_h = block_ops(h, h_dag, dh, dh_dag, n)
    psi = np.concatenate([np.zeros(n, dtype=np.complex128), b.ravel()])
    phi = block_left_start(psi, n, rule)
    y, L = krylov_sign(op, op_h, psi, phi, k, sign, tau)
    return y[:n], y[n:], L
