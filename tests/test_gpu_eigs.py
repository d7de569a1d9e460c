"""GPU eigensolver for the deflation data (ovd_compute_deflation) against the
oracle's dense eigendecomposition: eigenvalues, eigenvector residuals,
biorthonormality, the rank-one projector derivative of every derivative pair,
and the deflated derivative against the dense result."""
import numpy as np
import pytest

import synth
from oracle import deflation, dirac, matfun

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = (4, 4, 4, 4)   # N = 3072
MU = 0.3


@pytest.fixture(scope="module")
def dense():
    U = synth.make_links(DIMS, 0.5, 701)
    H = dirac.dense_h(U, DIMS, MU)
    dH = dirac.dense_dh_dmu(U, DIMS, MU)
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, 24)
    return U, H, dH, lam, R, L, dR, dL


def _flat(t):
    from gpu_helpers import host
    a = host(t)
    return a.reshape(a.shape[0], -1).T          # columns


def test_eigenpairs_and_derivatives(dense):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    U, H, dH, lam_o, R_o, L_o, dR_o, dL_o = dense
    m, l = 15, 4     # |lambda_15| = 0.543, |lambda_16| = 0.566: a gap, no cluster cut
    print_case(test="eigs", dims=DIMS, m=m, l=l)
    lat = ovderiv.Lattice(DIMS)
    lat.set_links(dev(U))
    lam, st = lat.compute_deflation(MU, m, l)
    print("eigensolver stats", st)
    assert st["max_res_right"] <= 1e-10 and st["max_res_left"] <= 1e-10
    assert st["max_biorth"] <= 1e-10
    # the same eigenvalues as the dense decomposition, in the same |lambda| order
    assert np.abs(lam - lam_o[:m]).max() < 1e-10
    lam2, Rt, Lt, dRt, dLt = lat.get_deflation(MU)
    assert np.array_equal(lam2, lam)
    R, L, dR, dL = _flat(Rt), _flat(Lt), _flat(dRt), _flat(dLt)
    assert np.abs(H @ R - R * lam).max() < 1e-9
    assert np.abs(np.conj(L).T @ H - lam[:, None] * np.conj(L).T).max() < 1e-9
    assert np.abs(np.conj(L).T @ R - np.eye(m)).max() < 1e-10
    # d/dmu of each rank-one spectral projector R_j L_j^dag is gauge free
    for j in range(l):
        dp = np.outer(dR[:, j], np.conj(L[:, j])) + np.outer(R[:, j], np.conj(dL[:, j]))
        dp_o = np.outer(dR_o[:, j], np.conj(L_o[:, j])) + np.outer(R_o[:, j], np.conj(dL_o[:, j]))
        assert np.abs(dp - dp_o).max() < 1e-8 * max(1.0, np.abs(dp_o).max()), j
        # gauge of the formula: L_j^dag dR_j = 0 = dL_j^dag R_j
        assert abs(np.vdot(L[:, j], dR[:, j])) < 1e-9 and abs(np.vdot(dL[:, j], R[:, j])) < 1e-9


def test_deflated_derivative_with_gpu_eigenpairs():
    """Generalised deflation (eq. 9-11) with GPU-computed eigen-data against the
    oracle's deflated derivative with its own dense eigen-data (the deflated
    result depends only on the spectral projectors and their derivatives, not
    on the eigenvector normalisation), and on rough links (eps = 1.0, small
    gap) a better result than the undeflated run at the same k."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, ops, print_case, rel
    dims, m, l, k = (4, 2, 2, 4), 16, 10, 96   # oracle, dense eigen-data: 0.35 -> 0.13
    print_case(test="eigs_deflated", dims=dims, m=m, l=l, k=k)
    U = synth.make_links(dims, 1.0, 301)
    b = synth.make_sources(dims, 1, 702)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    _, dy0, _ = lat.sign_apply_deriv(dev(b), MU, k)
    lam, st = lat.compute_deflation(MU, m, l)
    print("eigensolver stats", st, flush=True)
    _, dy1, _ = lat.sign_apply_deriv(dev(b), MU, k)
    lat.close()
    H = dirac.dense_h(U, dims, MU)
    dH = dirac.dense_dh_dmu(U, dims, MU)
    lam_o, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, m)
    assert np.abs(lam - lam_o).max() < 1e-10
    h, hd, dh, dhd = ops(U, dims, MU)
    dref, _, _ = deflation.deflate_gen(h, hd, dh, dhd, b[0].ravel(), k, lam_o[:l], R[:, :l], L[:, :l],
                                       dR[:, :l], dL[:, :l])
    assert rel(host(dy1)[0], dref) < 1e-9
    exact = matfun.frechet_sign_dd(H, dH) @ b[0].ravel()
    e0, e1 = rel(host(dy0)[0], exact), rel(host(dy1)[0], exact)
    print(f"derivative error at k={k}: undeflated {e0:.2e}, deflated (m={m}, l={l}) {e1:.2e}")
    assert e1 < 0.5 * e0
