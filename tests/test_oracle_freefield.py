"""Pins of the free-field closed form (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import dirac, freefield, matfun

MU = 0.3


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 2)])
def test_free_sign_matches_dense(dims):
    V = int(np.prod(dims))
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    b = synth.make_source(dims, 51).ravel()
    H = dirac.dense_h(U, dims, MU)
    dH = dirac.dense_dh_dmu(U, dims, MU)
    y, dy = freefield.sign_apply(b, dims, MU, deriv=True)
    assert np.abs(y - matfun.sign_schur(H) @ b).max() < 1e-12
    assert np.abs(dy - matfun.frechet_sign_block(H, dH) @ b).max() < 1e-11


def test_gauge_rotated_free_field():
    """Pure-gauge links: sgn(H[U_g]) b = G sgn(H[1]) G^dag b (random-looking links, known answer)."""
    dims = (2, 2, 2, 4)
    U, g = synth.gauge_rotated_unit_links(dims, 52)
    b = synth.make_source(dims, 53)
    H = dirac.dense_h(U, dims, MU)
    ref = matfun.sign_schur(H) @ b.ravel()
    gb = np.einsum("vba,vsb->vsa", np.conj(g), b)      # G^dag b
    y = freefield.sign_apply(gb.ravel(), dims, MU).reshape(-1, 4, 3)
    y = np.einsum("vab,vsb->vsa", g, y)
    assert np.abs(y.ravel() - ref).max() < 1e-12
