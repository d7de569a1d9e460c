"""Exact sgn(H(mu)) b and its mu-derivative for unit links -- oracle (test infrastructure only).

With U = 1 the kernel of eq. 1 is diagonal in momentum space.  For a plane
wave psi(x) = e^{i p.x} chi the hops of Dw(mu) multiply by e^{+-i p_nu}, and
the chemical potential enters as p_4 -> p_4 - i mu, so

    Dw(p) = m0 + 4r - r sum_nu cos(pt_nu) + i sum_nu gamma_nu sin(pt_nu),
    pt_k = p_k = 2 pi n_k / L_k (periodic space),
    pt_4 = p_4 - i mu,  p_4 = (2 n_4 + 1) pi / L_t (antiperiodic time),

and H(p) = gamma5 Dw(p) is a 4x4 spin matrix (times the colour identity).
sgn(H) b is then one 4x4 matrix sign per momentum, applied to the Fourier
transform of b; the derivative in mu is the top-right block of the sign of
the 8x8 block matrix [[H(p), dH(p)/dmu], [0, H(p)]] (eq. 6).  This gives exact
references at any lattice size.

Pinned by (tests/test_oracle_freefield.py): agreement with the dense sign of
the position-space operator on small lattices, and H(p) eigenvalues against the
dense spectrum.
"""
from __future__ import annotations

import numpy as np

from . import dirac, matfun


def momenta(dims):
    Lx, Ly, Lz, Lt = dims
    px = 2 * np.pi * np.arange(Lx) / Lx
    py = 2 * np.pi * np.arange(Ly) / Ly
    pz = 2 * np.pi * np.arange(Lz) / Lz
    pt = (2 * np.arange(Lt) + 1) * np.pi / Lt
    return px, py, pz, pt


def h_of_p(dims, mu, m0=-1.5, r=1.0):
    """H(p) and dH/dmu(p), arrays (Lt, Lz, Ly, Lx, 4, 4)."""
    px, py, pz, pt = momenta(dims)
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    ptil = [PX, PY, PZ, PT - 1j * mu]
    I4 = np.eye(4)
    D = (m0 + 4 * r) * I4 + 0 * PX[..., None, None]
    dD = np.zeros_like(D)
    for nu in range(4):
        D = D - r * np.cos(ptil[nu])[..., None, None] * I4 + 1j * np.sin(ptil[nu])[..., None, None] * dirac.GAMMA[nu]
    # d/dmu of -r cos(p4 - i mu) + i gamma4 sin(p4 - i mu)
    dD = dD + (-r * 1j * np.sin(ptil[3]))[..., None, None] * I4 + (np.cos(ptil[3]))[..., None, None] * dirac.GAMMA[3]
    H = np.einsum("st,...tu->...su", dirac.GAMMA5, D)
    dH = np.einsum("st,...tu->...su", dirac.GAMMA5, dD)
    return H, dH


def _to_momentum(b, dims):
    Lx, Ly, Lz, Lt = dims
    f = np.asarray(b).reshape(Lt, Lz, Ly, Lx, 4, 3)
    t = np.arange(Lt)
    tw = np.exp(-1j * np.pi * t / Lt)[:, None, None, None, None, None]
    return np.fft.fftn(f * tw, axes=(0, 1, 2, 3))


def _from_momentum(bt, dims):
    Lx, Ly, Lz, Lt = dims
    t = np.arange(Lt)
    tw = np.exp(1j * np.pi * t / Lt)[:, None, None, None, None, None]
    return np.fft.ifftn(bt, axes=(0, 1, 2, 3)) * tw


def sign_apply(b, dims, mu, m0=-1.5, r=1.0, deriv=False):
    """Exact sgn(H(mu)) b for U = 1 (flat [V*12]); with deriv=True also d/dmu of it."""
    H, dH = h_of_p(dims, mu, m0, r)
    bt = _to_momentum(b, dims)
    shp = H.shape[:4]
    S = np.empty_like(H)
    dS = np.empty_like(H) if deriv else None
    for idx in np.ndindex(*shp):
        if deriv:
            blk = matfun.sign_schur(matfun.block(H[idx], dH[idx]))
            S[idx] = blk[4:, 4:]
            dS[idx] = blk[:4, 4:]
        else:
            S[idx] = matfun.sign_schur(H[idx])
    y = _from_momentum(np.einsum("...st,...tc->...sc", S, bt), dims).reshape(-1)
    if not deriv:
        return y
    dy = _from_momentum(np.einsum("...st,...tc->...sc", dS, bt), dims).reshape(-1)
    return y, dy


def spectrum(dims, mu, m0=-1.5, r=1.0):
    """All eigenvalues of H(mu) for U = 1 (each 3-fold colour degenerate)."""
    H, _ = h_of_p(dims, mu, m0, r)
    ev = np.linalg.eigvals(H.reshape(-1, 4, 4)).ravel()
    return np.repeat(ev, 3)
