"""Gradient of s = <x|sgn(H)|b> w.r.t. mu and every link -- oracle (test infrastructure only).

The paper motivates derivatives of the overlap operator by conserved currents
and the fermionic force (Sec. 1) and computes the derivative along one
direction t with eq. 6-7.  The gradient with respect to all link parameters at
once follows from the same Frechet derivative: with K = L_sgn(H, b x^dag),

    ds/dt = x^dag L_sgn(H, dH/dt) b = tr(K dH/dt),

using tr(X L_f(A, E)) = tr(L_f(A, X) E).  By eq. 6, K is the top-right block
of sgn([[H, b x^dag], [0, H]]).

Krylov form (two-sided Lanczos with right start b and left start x):
b x^dag = (x^dag b) v_1 w_1^dag, so K ~ (x^dag b) V_k M_k W_k^dag with
M_k = L_sgn(T_k, e_1 e_1^T), the top-right block of sgn([[T_k, e_1 e_1^T], [0, T_k]]);
s ~ (x^dag b) [sgn(T_k)]_11 and ds/dt ~ (x^dag b) sum_p z_p^dag (dH/dt) v_p with Z = W_k M_k^dag.

Link force: for U_nu(y) -> exp(t X) U_nu(y) (dU = X U, dU^dag = -U^dag X) the
derivative is ds/dt = tr(F_nu(y) X) with

    F_nu(y) = -1/2 c_f s_f U_nu(y) Kf  +  1/2 c_b s_b Kb U_nu(y)^dag,
    Kf[b][a] = sum_{s,s'} (gamma5 (r - gamma_nu))_{s s'} K(y+nu, y)[s' b][s a],
    Kb[b][a] = sum_{s,s'} (gamma5 (r + gamma_nu))_{s s'} K(y, y+nu)[s' b][s a],

c_f = e^{mu}, c_b = e^{-mu} for nu = t (else 1), s_f, s_b the time-boundary
signs of the two hops.  The su(3) component along i lambda_a/2 is
tr(F i lambda_a/2); a U(1) phase exp(i theta) on the link gives i tr F
(``u1_derivative``), the derivative along the external U(1) field that Sec. 4
differentiates along.

Deflated form (``krylov_vjp_deflated``, with the eigenpairs of Sec. 3): the
Frechet kernel split over the deflated set and its complement (see there).

Pinned by (tests/test_oracle_vjp.py): central finite differences of s computed
with the dense sign, for mu and for random link directions; the Krylov form
against the dense K at large k; the deflated form against the dense gradient,
converging faster than the undeflated form on a small-gap field.
"""
from __future__ import annotations

import numpy as np

from . import dirac, matfun, tsl


def dense_K(H, b, x, method=matfun.sign_schur):
    """K = L_sgn(H, b x^dag), top-right block of sgn([[H, b x^dag], [0, H]])."""
    return matfun.frechet_sign_block(H, np.outer(b, np.conj(x)), method)


def force_from_K(K, U, dims, mu, r=1.0, bc_t=-1.0):
    """Per-link 3x3 matrices F_nu(y), shape [4][V][3][3], from a dense K (N x N)."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    Kb = K.reshape(V, 4, 3, V, 4, 3)
    U = np.asarray(U).reshape(4, V, 3, 3)
    F = np.zeros((4, V, 3, 3), dtype=np.complex128)
    coords = np.array(np.unravel_index(np.arange(V), (Lt, Lz, Ly, Lx)))  # t, z, y, x
    for nu in range(4):
        ax = 3 - nu                      # coordinate row of direction nu
        L = (Lx, Ly, Lz, Lt)[nu]
        c_f, c_b = (np.exp(mu), np.exp(-mu)) if nu == 3 else (1.0, 1.0)
        A_f = dirac.GAMMA5 @ (r * np.eye(4) - dirac.GAMMA[nu])
        A_b = dirac.GAMMA5 @ (r * np.eye(4) + dirac.GAMMA[nu])
        for y in range(V):
            c = coords[:, y].copy()
            wrap = c[ax] == L - 1
            c[ax] = (c[ax] + 1) % L
            yp = np.ravel_multi_index(tuple(c), (Lt, Lz, Ly, Lx))
            sgn = bc_t if (nu == 3 and wrap) else 1.0
            Kf = np.einsum("st,tbsa->ba", A_f, Kb[yp, :, :, y, :, :])
            Kbk = np.einsum("st,tbsa->ba", A_b, Kb[y, :, :, yp, :, :])
            F[nu, y] = (-0.5 * c_f * sgn) * (U[nu, y] @ Kf) + (0.5 * c_b * sgn) * (Kbk @ np.conj(U[nu, y]).T)
    return F


def dense_vjp(U, dims, mu, x, b, m0=-1.5, r=1.0, bc_t=-1.0):
    """(s, ds/dmu, F) from dense linear algebra (tiny lattices)."""
    H = dirac.dense_h(U, dims, mu, m0, r, bc_t)
    dH = dirac.dense_dh_dmu(U, dims, mu, r, bc_t)
    x = x.ravel()
    b = b.ravel()
    s = np.vdot(x, matfun.sign_schur(H) @ b)
    K = dense_K(H, b, x)
    ds_dmu = np.trace(K @ dH)
    F = force_from_K(K, U, dims, mu, r, bc_t)
    return s, ds_dmu, F


def krylov_vjp(U, dims, mu, x, b, k, m0=-1.5, r=1.0, bc_t=-1.0, tau=1e-14):
    """(s, ds/dmu, F, lanczos info) from the two-sided Lanczos form with right start b, left x."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0, r, bc_t))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0, r, bc_t))
    L = tsl.lanczos(h, hd, b, x, k, tau)
    T = L["T"]
    xb = np.vdot(x, b)
    s = xb * matfun.sign_schur(T)[0, 0]
    E = np.zeros_like(T)
    E[0, 0] = 1.0
    M = matfun.frechet_sign_block(T, E)
    Z = L["W"] @ np.conj(M).T
    dHV = np.stack([dirac.flat(dirac.apply_dh_dmu(U, L["V"][:, p], dims, mu, r, bc_t))
                    for p in range(k)], axis=1)
    ds_dmu = xb * np.sum(np.conj(Z) * dHV)
    # K_k = xb * sum_p v_p z_p^dag, assembled per link without forming N x N
    F = force_from_pairs(L["V"], Z, U, dims, mu, r, bc_t) * xb
    return s, ds_dmu, F, L


def krylov_vjp_deflated(U, dims, mu, x, b, k, lam, R, L, m0=-1.5, r=1.0, bc_t=-1.0, tau=1e-14):
    """(s, ds/dmu, F) with the m eigenpairs (lam, R, L; L^dag R = 1) deflated (Sec. 3, eq. 8).

    With P = sum_i R_i L_i^dag (set D) and Pbar = 1 - P, split the Frechet
    kernel K = L_sgn(H, b x^dag) = sum_{i,j} f[l_i, l_j] P_i b x^dag P_j
    (f[a, c] = (sgn a - sgn c)/(a - c), zero for equal signs) by whether i, j
    lie in D or in its complement C:
      K_CC = L_sgn(H, b' x'^dag), b' = Pbar b, x' = Pbar^dag x: the bilinear
             Krylov form with right start b' and left start x';
      K_CD = sum_{j in D} g_j(H) b' (x^dag R_j) L_j^dag,
      K_DC = sum_{i in D} (L_i^dag b) R_i x'^dag g_i(H),
             g_j(z) = (sgn z - s_j)/(z - l_j), whose Krylov-Ritz forms are
             |b'| V_k g_j(T_k) e_1 and (x'^dag v_1) e_1^T g_i(T_k) W_k^dag;
      K_DD = sum_{i,j in D} f[l_i, l_j] (L_i^dag b)(x^dag R_j) R_i L_j^dag, exact.
    s = x'^dag sgn(H) b' + sum_i s_i (x^dag R_i)(L_i^dag b).  All parts enter
    ds/dt = tr(K dH/dt) as pairs K = sum_p v_p z_p^dag.
    """
    x = np.asarray(x, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    lam = np.asarray(lam)
    Lh = np.conj(L).T
    Rh = np.conj(R).T
    c = Lh @ b                      # L_i^dag b
    d = Rh @ x                      # R_i^dag x, so x^dag R_i = conj(d_i)
    bp = b - R @ c
    xp = x - L @ d
    sg = matfun.sgn_scalar(lam)
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0, r, bc_t))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0, r, bc_t))
    Lz = tsl.lanczos(h, hd, bp, xp, k, tau)
    T, V, W = Lz["T"], Lz["V"], Lz["W"]
    kk = T.shape[0]
    xb = np.vdot(xp, bp)
    S = matfun.sign_schur(T)
    s = xb * S[0, 0] + np.sum(sg * np.conj(d) * c)
    E = np.zeros_like(T)
    E[0, 0] = 1.0
    M = matfun.frechet_sign_block(T, E)
    e1 = np.zeros(kk, dtype=np.complex128)
    e1[0] = 1.0
    I = np.eye(kk)
    nb = Lz["norm"]                          # |b'|
    x1 = np.vdot(xp, V[:, 0])                # x'^dag v_1
    vs, zs = [V], [W @ np.conj(M).T * np.conj(xb)]   # K_CC: xb V M W^dag
    m = lam.size
    A = np.empty((V.shape[0], m), dtype=np.complex128)
    Zi = np.zeros((V.shape[0], m), dtype=np.complex128)
    for j in range(m):
        gj = np.linalg.solve(T - lam[j] * I, S[:, 0] - sg[j] * e1)        # g_j(T) e_1
        A[:, j] = nb * np.conj(d[j]) * (V @ gj)
        rj = np.linalg.solve((T - lam[j] * I).T, S[0, :] - sg[j] * e1)    # (e_1^T g_j(T))^T
        Zi[:, j] += np.conj(c[j] * x1) * (W @ np.conj(rj))
    for i in range(m):
        for j in range(m):
            if sg[i] != sg[j]:
                fij = (sg[i] - sg[j]) / (lam[i] - lam[j])
                Zi[:, i] += np.conj(fij * c[i] * np.conj(d[j])) * L[:, j]
    vs += [A, R]
    zs += [L, Zi]
    Vall = np.concatenate(vs, axis=1)
    Zall = np.concatenate(zs, axis=1)
    dHV = np.stack([dirac.flat(dirac.apply_dh_dmu(U, Vall[:, p], dims, mu, r, bc_t))
                    for p in range(Vall.shape[1])], axis=1)
    ds_dmu = np.sum(np.conj(Zall) * dHV)
    F = force_from_pairs(Vall, Zall, U, dims, mu, r, bc_t)
    return s, ds_dmu, F, Lz


def force_from_pairs(Vb, Z, U, dims, mu, r=1.0, bc_t=-1.0):
    """F for K = sum_p v_p z_p^dag (columns of Vb and Z), link by link."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    k = Vb.shape[1]
    vf = Vb.T.reshape(k, V, 4, 3)
    zf = Z.T.reshape(k, V, 4, 3)
    U = np.asarray(U).reshape(4, V, 3, 3)
    F = np.zeros((4, V, 3, 3), dtype=np.complex128)
    coords = np.array(np.unravel_index(np.arange(V), (Lt, Lz, Ly, Lx)))
    for nu in range(4):
        ax = 3 - nu
        L = (Lx, Ly, Lz, Lt)[nu]
        c = coords.copy()
        wrap = c[ax] == L - 1
        c[ax] = (c[ax] + 1) % L
        yp = np.ravel_multi_index(tuple(c), (Lt, Lz, Ly, Lx))
        sgn = np.where(wrap & (nu == 3), bc_t, 1.0)
        c_f, c_b = (np.exp(mu), np.exp(-mu)) if nu == 3 else (1.0, 1.0)
        A_f = dirac.GAMMA5 @ (r * np.eye(4) - dirac.GAMMA[nu])
        A_b = dirac.GAMMA5 @ (r * np.eye(4) + dirac.GAMMA[nu])
        # K(y+nu, y)[s'b][sa] = sum_p v_p(y+nu)[s'b] conj(z_p(y)[sa])
        Kf = np.einsum("st,pytb,pysa->yba", A_f, vf[:, yp], np.conj(zf))
        Kb = np.einsum("st,pytb,pysa->yba", A_b, vf, np.conj(zf[:, yp]))
        F[nu] = ((-0.5 * c_f) * sgn)[:, None, None] * np.einsum("yab,ybc->yac", U[nu], Kf) \
            + ((0.5 * c_b) * sgn)[:, None, None] * np.einsum("yab,ycb->yac", Kb, np.conj(U[nu]))
    return F


def u1_derivative(F):
    """ds/dTheta_nu(y) = i tr F_nu(y) for the U(1) phases U_nu(y) -> e^{i Theta} U_nu(y), shape [4][V]."""
    return 1j * np.einsum("nvaa->nv", F)


def directional(F, X):
    """ds/dt = sum_links tr(F X) for a link-algebra direction X (dU = X U)."""
    return np.einsum("nvab,nvba->", F, X)
