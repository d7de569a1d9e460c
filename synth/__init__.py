"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws inputs only: SU(3) gauge links, complex Gaussian sources and
su(3) tangent directions.  It contains none of the method's arithmetic (no
Dirac operator, no Krylov step, no matrix function), so that the CPU oracle and
the GPU path can both be fed the same data without sharing any computation.

Layouts (complex128, C order), matching the C ABI of the library:
  * lattice ``dims = (Lx, Ly, Lz, Lt)``; site index ``x + Lx*(y + Ly*(z + Lz*t))``;
  * spinor field ``[V][4][3]`` (spin, colour);
  * link field ``[4][V][3][3]`` with direction order x, y, z, t.

The paper's ensembles (quenched Luescher-Weisz configurations on 14x14^3 and
6x18^3, Sec. 4) are not available; links here are random SU(3) matrices
``exp(i*eps*sum_a c_a lambda_a/2)`` with ``c_a ~ N(0,1)`` drawn from a seed,
followed by reunitarisation.  Small ``eps`` gives a smooth field whose Wilson
kernel has a wide spectral gap around zero, like the paper's high-temperature
ensemble.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann", "volume", "make_links", "reunitarize", "make_source",
    "make_sources", "make_su3_direction", "make_gauge_rotation",
    "gauge_rotated_unit_links", "LATTICES",
]

# Lattice shapes of the workloads, (Lx, Ly, Lz, Lt).
LATTICES = {
    "2^4": (2, 2, 2, 2),
    "4^4": (4, 4, 4, 4),
    "6^4": (6, 6, 6, 6),
    "8^4": (8, 8, 8, 8),
    "10^4": (10, 10, 10, 10),
    "12^4": (12, 12, 12, 12),
    "14x14^3": (14, 14, 14, 14),
    "16^4": (16, 16, 16, 16),
    "20x20^3": (20, 20, 20, 20),
}


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def reunitarize(U: np.ndarray) -> np.ndarray:
    """Project 3x3 matrices back to SU(3): Gram-Schmidt on rows 1-2, row 3 = conj(r1 x r2)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    r1 = U[..., 0, :]
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = U[..., 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1, keepdims=True) * r1
    r2 = r2 / np.linalg.norm(r2, axis=-1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=-2)


def _expi_hermitian(A: np.ndarray) -> np.ndarray:
    """exp(i A) for a stack of Hermitian 3x3 matrices, via eigendecomposition."""
    w, Q = np.linalg.eigh(A)
    return np.einsum("...ij,...j,...kj->...ik", Q, np.exp(1j * w), np.conj(Q))


def make_links(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) link field ``[4][V][3][3]``.

    ``U_nu(x) = exp(i*eps*sum_a c_a lambda_a / 2)`` with ``c_a ~ N(0,1)``; the
    draws are ordered site-lexicographic, then direction, then generator, from
    numpy's PCG64 seeded with ``seed``.
    """
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.standard_normal((V, 4, 8))
    lam = gell_mann()
    A = 0.5 * eps * np.einsum("vna,aij->nvij", c, lam)
    return np.ascontiguousarray(reunitarize(_expi_hermitian(A)))


def make_source(dims, seed: int) -> np.ndarray:
    """Complex Gaussian spinor ``[V][4][3]``, normalised to unit 2-norm."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = (rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))) / np.sqrt(2.0)
    return np.ascontiguousarray(z / np.linalg.norm(z))


def make_sources(dims, n: int, seed: int) -> np.ndarray:
    """``n`` unit sources ``[n][V][4][3]``; source i uses seed ``seed + i``."""
    return np.stack([make_source(dims, seed + i) for i in range(n)])


def make_su3_direction(dims, seed: int) -> np.ndarray:
    """Random su(3) tangent field ``X_nu(x) = i*sum_a eta_a lambda_a/2``, ``eta_a ~ N(0,1)``.

    Returned as ``[4][V][3][3]`` anti-Hermitian traceless matrices.  The link
    derivative direction used by the library is ``dU = X U``.
    """
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    eta = rng.standard_normal((V, 4, 8))
    lam = gell_mann()
    return np.ascontiguousarray(0.5j * np.einsum("vna,aij->nvij", eta, lam))


def make_gauge_rotation(dims, seed: int) -> np.ndarray:
    """Random SU(3) matrices ``g(x)``, shape ``[V][3][3]`` (Haar-like via QR)."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = (rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q[:, :, 0] = Q[:, :, 0] / det[:, None]
    return np.ascontiguousarray(Q)


def gauge_rotated_unit_links(dims, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Pure-gauge links ``U_nu(x) = g(x) g(x+nu)^dag`` and the rotation ``g``.

    Periodic in every direction (the time boundary sign lives in the stencil,
    not in the links), so the Dirac operator on these links is the free one
    conjugated by ``g``.
    """
    Lx, Ly, Lz, Lt = dims
    g = make_gauge_rotation(dims, seed)
    g5 = g.reshape(Lt, Lz, Ly, Lx, 3, 3)
    U = np.empty((4, Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    for nu, ax in enumerate((3, 2, 1, 0)):
        gp = np.roll(g5, -1, axis=ax)
        U[nu] = np.einsum("...ab,...cb->...ac", g5, np.conj(gp))
    return np.ascontiguousarray(U.reshape(4, -1, 3, 3)), g
