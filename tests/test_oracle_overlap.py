"""Pins of the oracle's overlap operator (eq. 1), no GPU."""
import numpy as np

import synth
from oracle import overlap

DIMS = (2, 2, 2, 2)


def test_ginsparg_wilson_relation():
    U = synth.make_links(DIMS, 0.5, 61)
    for mu in (0.0, 0.3):
        D = overlap.dense_overlap(U, DIMS, mu)
        G5 = overlap.gamma5_field(D.shape[0])
        assert np.abs(G5 @ D + D @ G5 - D @ G5 @ D).max() < 1e-10


def test_circle_and_gamma5_hermiticity_at_zero_mu():
    U = synth.make_links(DIMS, 0.5, 62)
    D = overlap.dense_overlap(U, DIMS, 0.0)
    G5 = overlap.gamma5_field(D.shape[0])
    lam = np.linalg.eigvals(D)
    assert np.abs(np.abs(lam - 1.0) - 1.0).max() < 1e-10
    assert np.abs(D.conj().T - G5 @ D @ G5).max() < 1e-10


def test_krylov_overlap_converges_to_dense():
    U = synth.make_links(DIMS, 0.5, 63)
    b = synth.make_source(DIMS, 64).ravel()
    D = overlap.dense_overlap(U, DIMS, 0.3)
    errs = [np.linalg.norm(overlap.krylov_overlap(U, DIMS, 0.3, b, k) - D @ b) for k in (40, 120, 180)]
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-6
