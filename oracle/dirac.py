"""Wilson-Dirac kernel at chemical potential -- oracle (test infrastructure only).

Sec. 1, eq. 1: the overlap operator uses the kernel H(mu) = gamma5 Dw(mu), with
Dw(mu) the Wilson-Dirac operator at quark chemical potential mu.  The paper does
not print Dw; this module uses the standard exponential prescription:

  Dw(mu) psi(x) = (m0 + 4 r) psi(x)
      - 1/2 sum_{nu=1..4} [ e^{+mu d_nu4} (r - gamma_nu) U_nu(x)        psi(x + nu)
                           + e^{-mu d_nu4} (r + gamma_nu) U_nu(x - nu)^dag psi(x - nu) ]

periodic in space, antiperiodic in time (a factor -1 on the hops that cross
t = Lt-1 <-> 0, kept out of the links), chiral gamma basis
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]], so
gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1); spinor index
3*spin + colour.

Derivatives (Sec. 2, the derivative direction t):
  * t = mu: only the temporal hops depend on mu;
  * t = a link parameter with tangent dU_nu(x) = d U_nu(x)/dt: the hopping
    term with U replaced by dU (and U^dag by dU^dag), no mass term.

The operator is applied with numpy rolls and einsums, one direction at a time,
exactly as the formula reads.  Fields carry optional leading batch axes.

Pinned by (tests/test_oracle_dirac.py): anticommutation of the gamma matrices,
H(mu)^dag = H(-mu) for every link field, H(0) Hermitian, gauge covariance,
the free-field momentum-space spectrum, and finite differences for both
derivatives.
"""
from __future__ import annotations

import numpy as np

# --- gamma matrices (chiral basis) -----------------------------------------
_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)

GAMMA = np.stack(
    [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in (_s1, _s2, _s3)]
    + [np.block([[_Z2, _I2], [_I2, _Z2]])]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

# lattice axis of direction nu in a field shaped (..., Lt, Lz, Ly, Lx, 4, 3)
_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


def as_field(psi, dims):
    """Reshape ``[..., V, 4, 3]`` (or flat ``[..., 12V]``) to ``(..., Lt, Lz, Ly, Lx, 4, 3)``."""
    Lx, Ly, Lz, Lt = dims
    psi = np.asarray(psi)
    if psi.ndim >= 6 and psi.shape[-6:] == (Lt, Lz, Ly, Lx, 4, 3):
        return psi
    lead = psi.shape[:-1] if psi.shape[-1] == 12 * Lx * Ly * Lz * Lt else psi.shape[:-3]
    return psi.reshape(lead + (Lt, Lz, Ly, Lx, 4, 3))


def as_links(U, dims):
    Lx, Ly, Lz, Lt = dims
    return np.asarray(U).reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def flat(psi_field):
    """``(..., Lt, Lz, Ly, Lx, 4, 3)`` -> ``(..., 12V)``."""
    lead = psi_field.shape[:-6]
    return psi_field.reshape(lead + (-1,))


def _spin(G, psi):
    return np.einsum("st,...ta->...sa", G, psi)


def _colour(U, psi):
    # U: (Lt, Lz, Ly, Lx, 3, 3) acting on psi (..., Lt, Lz, Ly, Lx, 4, 3)
    return np.einsum("tzyxab,...tzyxsb->...tzyxsa", U, psi)


def _colour_dag(U, psi):
    return np.einsum("tzyxba,...tzyxsb->...tzyxsa", np.conj(U), psi)


def _shift(psi, nu, step, bc_t):
    """psi(x + step*nu), with the time boundary factor on hops crossing t=Lt-1<->0."""
    ax = _AXIS[nu]
    out = np.roll(psi, -step, axis=ax)
    if nu == 3 and bc_t != 1:
        out = np.array(out, copy=True)
        idx = [slice(None)] * out.ndim
        idx[ax] = -1 if step == 1 else 0
        out[tuple(idx)] *= bc_t
    return out


def hopping(U, psi, dims, mu, r=1.0, bc_t=-1.0, dmu=False):
    """Hopping part  -1/2 sum_nu [...]  of Dw(mu) (no mass term).

    With ``dmu=True`` returns its mu-derivative instead (temporal hops only,
    forward coefficient +e^{mu}, backward -e^{-mu}).  ``U`` may be any 3x3
    matrix field (e.g. a link tangent dU), unitarity is not assumed.
    """
    Uf = as_links(U, dims)
    psi = as_field(psi, dims)
    out = np.zeros(np.broadcast_shapes(psi.shape), dtype=np.complex128)
    for nu in range(4):
        if dmu and nu != 3:
            continue
        if nu == 3:
            cf, cb = np.exp(mu), np.exp(-mu)
            if dmu:
                cb = -cb
        else:
            cf = cb = 1.0
        Pm = r * np.eye(4) - GAMMA[nu]
        Pp = r * np.eye(4) + GAMMA[nu]
        fwd = _colour(Uf[nu], _shift(psi, nu, +1, bc_t))
        bwd = _shift(_colour_dag(Uf[nu], psi), nu, -1, bc_t)
        out = out - 0.5 * (cf * _spin(Pm, fwd) + cb * _spin(Pp, bwd))
    return out


def apply_dw(U, psi, dims, mu, m0=-1.5, r=1.0, bc_t=-1.0):
    """Dw(mu) psi; returns a field shaped like ``as_field(psi)``."""
    return (m0 + 4 * r) * as_field(psi, dims) + hopping(U, psi, dims, mu, r, bc_t)


def apply_h(U, psi, dims, mu, m0=-1.5, r=1.0, bc_t=-1.0):
    """H(mu) psi = gamma5 Dw(mu) psi (eq. 1)."""
    return _spin(GAMMA5, apply_dw(U, psi, dims, mu, m0, r, bc_t))


def apply_hdag(U, psi, dims, mu, m0=-1.5, r=1.0, bc_t=-1.0):
    """H(mu)^dag psi computed from the definition: Dw(mu)^dag gamma5 psi.

    The adjoint of each hop is written out (forward hop <-> backward hop with
    the Hermitian-conjugated link and spin factor), independent of the
    identity H(mu)^dag = H(-mu) that the tests check.
    """
    Uf = as_links(U, dims)
    phi = _spin(GAMMA5, as_field(psi, dims))
    out = np.conj(m0 + 4 * r) * phi
    for nu in range(4):
        cf, cb = (np.exp(mu), np.exp(-mu)) if nu == 3 else (1.0, 1.0)
        Pm = r * np.eye(4) - GAMMA[nu]
        Pp = r * np.eye(4) + GAMMA[nu]
        # adjoint of  x <- cf Pm U(x) phi(x+nu):   y+nu <- conj(cf) Pm^dag U(y)^dag phi(y)
        a_f = _shift(_colour_dag(Uf[nu], _spin(Pm.conj().T, phi)), nu, -1, bc_t)
        # adjoint of  x <- cb Pp U(x-nu)^dag phi(x-nu):   y-nu <- conj(cb) Pp^dag U(y-nu) phi(y)
        a_b = _colour(Uf[nu], _shift(_spin(Pp.conj().T, phi), nu, +1, bc_t))
        out = out - 0.5 * (np.conj(cf) * a_f + np.conj(cb) * a_b)
    return out


def apply_dh_dmu(U, psi, dims, mu, r=1.0, bc_t=-1.0):
    """(d/dmu H(mu)) psi = gamma5 d/dmu Dw(mu) psi."""
    return _spin(GAMMA5, hopping(U, psi, dims, mu, r, bc_t, dmu=True))


def apply_dh_dlink(dU, psi, dims, mu, r=1.0, bc_t=-1.0):
    """(d/dt H) psi for links moving along the tangent dU = dU/dt."""
    return _spin(GAMMA5, hopping(dU, psi, dims, mu, r, bc_t))


def dense(apply, N):
    """Dense matrix of a linear map on C^N by applying it to the unit vectors."""
    M = np.empty((N, N), dtype=np.complex128)
    eye = np.eye(N, dtype=np.complex128)
    step = 512
    for c0 in range(0, N, step):
        cols = eye[c0:c0 + step]
        M[:, c0:c0 + step] = np.asarray(apply(cols)).reshape(len(cols), N).T
    return M


def dense_h(U, dims, mu, m0=-1.5, r=1.0, bc_t=-1.0):
    N = 12 * int(np.prod(dims))
    return dense(lambda c: flat(apply_h(U, c, dims, mu, m0, r, bc_t)), N)


def dense_dh_dmu(U, dims, mu, r=1.0, bc_t=-1.0):
    N = 12 * int(np.prod(dims))
    return dense(lambda c: flat(apply_dh_dmu(U, c, dims, mu, r, bc_t)), N)


def dense_dh_dlink(dU, dims, mu, r=1.0, bc_t=-1.0):
    N = 12 * int(np.prod(dims))
    return dense(lambda c: flat(apply_dh_dlink(dU, c, dims, mu, r, bc_t)), N)


def link_tangent(X, U):
    """dU = X U for a link-algebra direction X (both ``[4][V][3][3]``)."""
    return np.einsum("nvab,nvbc->nvac", X, U)
