"""Pins of the oracle's nested two-sided Lanczos for sgn(T_k) e_1 (Sec. 4).

The nested run signs the outer Ritz matrix T by an inner Krylov-Ritz run on
Tt = (T + T^{-1}) / 2.  Checked here against facts outside the nested code:
  * sgn(Tt) = sgn(T) for dense matrices (the map z -> (z + 1/z)/2 keeps the
    sign of Re z), by the independent Schur and spectral signs;
  * at inner size kp = k the inner space is all of C^k: the result equals the
    Schur sign of T to rounding;
  * for the Ritz matrix of the 4^4 Wilson kernel the error against the Schur
    sign falls geometrically with kp (measured: 6e-6 at kp = 32, 1e-9 at 64,
    5e-14 at 100 for k = 128).
"""
import numpy as np

import synth
from oracle import dirac, matfun, tsl


def _random_tridiag(k, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    d = rng.choice([-1.0, 1.0], k) * rng.uniform(0.4, 3.0, k) + 0.3j * rng.standard_normal(k) + shift
    up = 0.4 * (rng.standard_normal(k - 1) + 1j * rng.standard_normal(k - 1))
    lo = 0.4 * rng.uniform(0.2, 1.0, k - 1)
    return np.diag(d) + np.diag(up, 1) + np.diag(lo, -1)


def test_joukowski_map_keeps_the_sign():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30))
    At = 0.5 * (A + np.linalg.inv(A))
    assert np.abs(matfun.sign_schur(At) - matfun.sign_schur(A)).max() < 1e-11
    assert np.abs(matfun.sign_eig(At) - matfun.sign_schur(A)).max() < 1e-9


def test_full_inner_size_is_exact():
    T = _random_tridiag(40, 12)
    ref = matfun.sign_schur(T)[:, 0]
    c = tsl.NestedSign(40)(T)
    assert np.linalg.norm(c - ref) < 1e-10 * np.linalg.norm(ref)
    # the inner size is clamped to k
    assert np.linalg.norm(tsl.NestedSign(60)(T) - ref) < 1e-10 * np.linalg.norm(ref)


def test_converges_in_inner_size_on_a_lattice_ritz_matrix():
    dims, mu = (4, 4, 4, 4), 0.3
    U = synth.make_links(dims, 0.5, 1)
    b = synth.make_source(dims, 2).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu))
    T = tsl.lanczos(h, hd, b, b, 128, keep_basis=False)["T"]
    ref = matfun.sign_schur(T)[:, 0]
    errs = [np.linalg.norm(tsl.NestedSign(kp)(T) - ref) / np.linalg.norm(ref) for kp in (16, 32, 64, 100)]
    assert all(a > 10 * b_ for a, b_ in zip(errs, errs[1:-1])), errs
    assert errs[2] < 1e-7 and errs[3] < 1e-11, errs


def test_nested_krylov_sign_matches_schur_variant_at_large_inner_size():
    """Through the whole Krylov-Ritz approximation: with the inner size at k the
    nested and the Schur variants of sgn(H) b agree to rounding."""
    dims, mu, k = (2, 2, 2, 4), 0.2, 40
    U = synth.make_links(dims, 0.5, 3)
    b = synth.make_source(dims, 4).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu))
    y1, _ = tsl.krylov_sign(h, hd, b, b, k)
    y2, _ = tsl.krylov_sign(h, hd, b, b, k, sign=tsl.NestedSign(k))
    assert np.linalg.norm(y1 - y2) < 1e-10 * np.linalg.norm(y1)
