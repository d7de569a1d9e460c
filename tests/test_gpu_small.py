"""The small dense step sgn(T_k) e_1 on the GPU (ovd_tridiag_sign and the
sign_method option) against the oracle.

  * the resolvent quadrature against the oracle's Schur-Sylvester sign on
    random complex tridiagonal matrices and on the Ritz matrix of a lattice
    operator, to 1e-10;
  * Ritz values close to the imaginary axis (where the sign jumps, Sec. 3):
    the quadrature needs more refinement levels there; with too few allowed
    levels the call fails with OVD_ENOCONV instead of returning an
    unconverged result, and with enough it matches the oracle;
  * the nested two-sided Lanczos of Sec. 4 against the oracle's NestedSign
    at equal inner size, directly and through a whole derivative call.
"""
import numpy as np
import pytest

import synth
from oracle import dirac, matfun, tsl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _split(T):
    """T (k x k tridiagonal) -> alpha, beta, delta in the library's convention."""
    k = T.shape[0]
    a = np.diag(T).copy()
    b = np.zeros(k, complex)
    d = np.zeros(k, complex)
    b[1:] = np.diag(T, 1)
    d[1:] = np.diag(T, -1)
    return a, b, d


def _random_tridiag(k, seed):
    rng = np.random.default_rng(seed)
    dg = rng.choice([-1.0, 1.0], k) * rng.uniform(0.4, 3.0, k) + 0.3j * rng.standard_normal(k)
    up = 0.4 * (rng.standard_normal(k - 1) + 1j * rng.standard_normal(k - 1))
    lo = 0.4 * rng.uniform(0.2, 1.0, k - 1)
    return np.diag(dg) + np.diag(up, 1) + np.diag(lo, -1)


def _lattice_ritz(k, seed=2):
    dims, mu = (4, 4, 4, 4), 0.3
    U = synth.make_links(dims, 0.5, 1)
    b = synth.make_source(dims, seed).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu))
    return tsl.lanczos(h, hd, b, b, k, keep_basis=False)["T"]


def test_quadrature_against_schur():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import print_case, rel
    Ts = [_random_tridiag(40, 1), _random_tridiag(40, 2), _lattice_ritz(40)]
    print_case(test="small_quad", k=40, nt=3)
    ab = [np.stack(x) for x in zip(*[_split(T) for T in Ts])]
    c, chk = ovderiv.tridiag_sign(*ab)
    for i, T in enumerate(Ts):
        assert rel(c[i], matfun.sign_schur(T)[:, 0]) < 1e-10, i
    assert chk <= 1e-10
    # a single large Ritz matrix
    T = _lattice_ritz(200, seed=3)
    print_case(test="small_quad", k=200, nt=1)
    c, _ = ovderiv.tridiag_sign(*[x[None] for x in _split(T)])
    assert rel(c[0], matfun.sign_schur(T)[:, 0]) < 1e-10


def test_eigenvalue_near_imaginary_axis_needs_levels_and_never_passes_silently():
    """T with an eigenvalue 5e-4 + 1i: the trapezoidal rule converges like
    exp(-2 pi d / h), d ~ 5e-4 the distance of its argument from pi/2, so four
    levels cannot reach 1e-10 and the call reports OVD_ENOCONV; fourteen can."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import print_case, rel
    k = 6
    T = np.diag([5e-4 + 1.0j, -0.6 + 0.1j, 1.2, -2.0 - 0.2j, 0.8 + 0.3j, -1.1]).astype(complex)
    T += np.diag([0.01, 0.2, 0.1, 0.3, 0.2], 1) + np.diag([0.02, 0.1, 0.2, 0.1, 0.15], -1)
    ab = [x[None] for x in _split(T)]
    print_case(test="small_near_axis", k=k, levels=4)
    with pytest.raises(ovderiv.OvdError) as ei:
        ovderiv.tridiag_sign(*ab, quad_max_levels=4)
    assert ei.value.status == ovderiv.OVD_ENOCONV and ei.value.check > 1e-10
    print_case(test="small_near_axis", k=k, levels=14)
    c, chk = ovderiv.tridiag_sign(*ab, quad_max_levels=14)
    assert chk <= 1e-10
    assert rel(c[0], matfun.sign_schur(T)[:, 0]) < 1e-9


@pytest.mark.parametrize("kp", [24, 64])
def test_nested_against_oracle_nested(kp):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import print_case, rel
    k = 128
    T = _lattice_ritz(k)
    print_case(test="small_nested", k=k, kp=kp)
    c, _ = ovderiv.tridiag_sign(*[x[None] for x in _split(T)], method=ovderiv.SIGN_NESTED, nested_inner=kp)
    ref = tsl.NestedSign(kp)(T)
    assert rel(c[0], ref) < 1e-10
    # and it approaches the full sign as kp grows (measured 9e-5 at 24, 1e-9 at 64)
    e = rel(c[0], matfun.sign_schur(T)[:, 0])
    assert e < (1e-3 if kp == 24 else 1e-8), e


def test_nested_sign_in_a_derivative_call():
    """sign_method = nested through the whole block-derivative pipeline (eq. 7)
    at 4^4, k = 64, inner size 40, against the oracle with the same nested sign."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, ops, print_case, rel
    dims, mu, k, kp = (4, 4, 4, 4), 0.3, 64, 40
    print_case(test="nested_deriv", dims=dims, k=k, kp=kp)
    U = synth.make_links(dims, 0.5, 1)
    b = synth.make_sources(dims, 2, 21)
    lat = ovderiv.Lattice(dims, sign_method=ovderiv.SIGN_NESTED, nested_inner=kp)
    lat.set_links(dev(U))
    y, dy, _ = lat.sign_apply_deriv(dev(b), mu, k)
    ys = host(lat.sign_apply(dev(b), mu, k))
    lat.close()
    h, hd, dh, dhd = ops(U, dims, mu)
    for r in range(2):
        dref, yref, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b[r].ravel(), k, sign=tsl.NestedSign(kp))
        assert rel(host(dy)[r], dref) < 1e-10
        assert rel(host(y)[r], yref) < 1e-10
        sref, _ = tsl.krylov_sign(h, hd, b[r].ravel(), b[r].ravel(), k, sign=tsl.NestedSign(kp))
        assert rel(ys[r], sref) < 1e-10
