"""GPU parity of the gradient of s = <x|sgn(H(mu))|b> (ovd_sign_apply_vjp, autograd).

Same-k parity against the oracle's Krylov VJP (same two-sided Lanczos, Frechet
derivative of sgn(T_k) by the Schur-Sylvester block method), convergence to
the dense gradient at large k, the autograd wrapper against central
finite differences of the oracle's dense <x|sgn(H)|b>, and
torch.autograd.gradcheck of the wrapper at a converged k.
"""
import numpy as np
import pytest

import synth
from oracle import dirac, matfun, vjp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MU = 0.3


def _lat(dims, U):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    return lat


@pytest.mark.parametrize("dims,k,eps", [((4, 2, 2, 4), 48, 0.5), ((4, 4, 4, 4), 96, 0.4), ((2, 2, 2, 2), 20, 1.0)])
def test_vjp_parity_same_k(dims, k, eps):
    from gpu_helpers import dev, host, print_case, rel
    print_case(test="vjp_same_k", dims=dims, k=k, eps=eps)
    U = synth.make_links(dims, eps, 501)
    x = synth.make_source(dims, 502)
    b = synth.make_source(dims, 503)
    s_r, dm_r, F_r, _ = vjp.krylov_vjp(U, dims, MU, x, b, k)
    lat = _lat(dims, U)
    s, dm, F, dU, dUc = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, force=True, wirtinger=True)
    assert abs(s - s_r) < 1e-10 * abs(s_r)
    assert abs(dm - dm_r) < 1e-10 * abs(dm_r)
    assert rel(host(F), F_r) < 1e-10
    # Wirtinger derivatives reproduce the force along any su(3) direction: dU = X U
    X = synth.make_su3_direction(dims, 504)
    E = np.einsum("nvab,nvbc->nvac", X, U)
    d_w = np.sum(host(dU) * E) + np.sum(host(dUc) * np.conj(E))
    d_f = vjp.directional(host(F), X)
    assert abs(d_w - d_f) < 1e-10 * max(1.0, abs(d_f))
    # s alone agrees with the value computed with the gradient
    s2, dm2, F2, _, _ = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, grad=False)
    assert dm2 is None and F2 is None and abs(s2 - s) < 1e-13 * abs(s)


def test_vjp_converges_to_dense():
    from gpu_helpers import dev, host, print_case
    dims = (2, 2, 2, 2)
    print_case(test="vjp_dense", dims=dims)
    U = synth.make_links(dims, 0.5, 41)
    x = synth.make_source(dims, 42)
    b = synth.make_source(dims, 43)
    s_d, dm_d, F_d = vjp.dense_vjp(U, dims, MU, x, b)
    lat = _lat(dims, U)
    errs = []
    for k in (40, 160):
        s, dm, F, _, _ = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k)
        errs.append((abs(s - s_d), abs(dm - dm_d), np.abs(host(F) - F_d).max()))
    assert errs[1][0] < 1e-12 and errs[1][1] < 1e-7 and errs[1][2] < 1e-8
    assert all(errs[1][i] < errs[0][i] for i in range(3))


def test_autograd_against_oracle_and_finite_differences():
    """L = Re(c s); torch gradients of U (complex), mu, x and b along random
    directions.  Parity: the oracle's Krylov gradient at the same k (1e-9).
    Exactness: central differences of the dense sign, which the GPU value must
    match as closely as the oracle's own Krylov value does (the truncation
    error at this k, 1e-3 for the bilinear and 3e-3 for the one-sided solves)."""
    from paper_1611_00195_amd.functional import sign_bilinear
    from gpu_helpers import dev, host, print_case
    from oracle import tsl
    dims, k = (2, 2, 2, 2), 64
    print_case(test="vjp_autograd", dims=dims, k=k)
    U = synth.make_links(dims, 0.5, 511)
    x = synth.make_source(dims, 512)
    b = synth.make_source(dims, 513)
    c = 0.7 - 0.4j
    from paper_1611_00195_amd import ovderiv
    lat = ovderiv.Lattice(dims)
    Ut, xt, bt = dev(U).requires_grad_(), dev(x).requires_grad_(), dev(b).requires_grad_()
    mut = torch.tensor(MU, dtype=torch.float64, requires_grad=True)
    s = sign_bilinear(lat, Ut, mut, xt, bt, k)
    (s * c).real.backward()

    def L(Uh, mu, xh, bh):
        S = matfun.sign_schur(dirac.dense_h(Uh, dims, mu))
        return (c * np.vdot(xh.ravel(), S @ bh.ravel())).real

    # oracle at the same k: K_k = (x^dag b) V_k M_k W_k^dag, and the one-sided
    # sgn(H(mu)) b and sgn(H(-mu)) x = sgn(H)^dag x
    ops = lambda mu: (lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu)),
                      lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu)))
    Lz = tsl.lanczos(*ops(MU), b.ravel(), x.ravel(), k)
    E1 = np.zeros_like(Lz["T"])
    E1[0, 0] = 1.0
    Kk = np.vdot(x.ravel(), b.ravel()) * Lz["V"] @ matfun.frechet_sign_block(Lz["T"], E1) @ np.conj(Lz["W"]).T
    Sb, _ = tsl.krylov_sign(*ops(MU), b.ravel(), b.ravel(), k)
    Sx, _ = tsl.krylov_sign(*ops(-MU), x.ravel(), x.ravel(), k)

    rng = np.random.default_rng(514)
    cn = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    h = 1e-5

    def check(an, kv, fd):
        an, kv, fd = float(an), float(kv), float(fd)
        assert abs(an - kv) < 1e-9 * max(1.0, abs(kv)), ("parity", an, kv)
        assert abs(an - fd) <= 1.5 * abs(kv - fd) + 1e-8, ("exactness", an, kv, fd)

    # complex, non-unitary link direction: dL = Re(sum conj(grad) E)
    E = cn(*U.shape)
    check(np.sum(np.conj(host(Ut.grad)) * E).real,
          (c * np.trace(Kk @ dirac.dense_dh_dlink(E, dims, MU))).real,
          (L(U + h * E, MU, x, b) - L(U - h * E, MU, x, b)) / (2 * h))
    check(mut.grad.item(), (c * np.trace(Kk @ dirac.dense_dh_dmu(U, dims, MU))).real,
          (L(U, MU + h, x, b) - L(U, MU - h, x, b)) / (2 * h))
    ex = cn(*x.shape)
    check(np.sum(np.conj(host(xt.grad)) * ex).real, (c * np.vdot(ex.ravel(), Sb)).real,
          (L(U, MU, x + h * ex, b) - L(U, MU, x - h * ex, b)) / (2 * h))
    eb = cn(*b.shape)
    check(np.sum(np.conj(host(bt.grad)) * eb).real, (c * np.vdot(Sx, eb.ravel())).real,
          (L(U, MU, x, b + h * eb) - L(U, MU, x, b - h * eb)) / (2 * h))


def test_autograd_gradcheck():
    """torch.autograd.gradcheck of sign_bilinear on 2^4 (complex output: real
    and imaginary parts checked separately), over U, mu, x and b together.
    At k = 160 the Krylov value has converged (1e-12 against the dense sign),
    so central differences of the forward are the exact gradient, which the
    library's VJP reproduces to ~1e-7 (test_vjp_converges_to_dense).  Fast
    mode: random projections u, v of the Jacobian, v^T J u numerically and
    analytically."""
    from paper_1611_00195_amd import ovderiv
    from paper_1611_00195_amd.functional import sign_bilinear
    from gpu_helpers import dev, print_case
    dims, k = (2, 2, 2, 2), 160
    print_case(test="vjp_gradcheck", dims=dims, k=k)
    torch.manual_seed(524)
    U = synth.make_links(dims, 0.5, 521)
    x = synth.make_source(dims, 522)
    b = synth.make_source(dims, 523)
    lat = ovderiv.Lattice(dims)
    inputs = (dev(U).requires_grad_(), torch.tensor(MU, dtype=torch.float64, requires_grad=True),
              dev(x).requires_grad_(), dev(b).requires_grad_())

    def fn(U_, mu_, x_, b_):
        return sign_bilinear(lat, U_, mu_, x_, b_, k)

    # eps = 1e-5 keeps the rounding noise of the converged forward (~1e-12)
    # below 1e-7 in the difference quotients
    assert torch.autograd.gradcheck(fn, inputs, eps=1e-5, atol=1e-5, rtol=1e-3, fast_mode=True)
    lat.close()


def test_vjp_dsdmu_agrees_with_block_derivative():
    """Two different GPU routes to d<x|sgn(H)|b>/dmu: the bilinear gradient
    (one Lanczos run with left start x, Frechet derivative of sgn(T_k)) and the
    block-matrix derivative of eq. 6-7 projected on x (storage-free mode).  On
    smooth links (eps = 0.4, as at the benchmark size) both have converged at
    k = 400 and must agree; the block route's own change from k = 300 to 400
    bounds its truncation error."""
    from gpu_helpers import dev, print_case
    dims = (6, 6, 6, 6)
    print_case(test="vjp_vs_block", dims=dims)
    U = synth.make_links(dims, 0.4, 521)
    x = synth.make_source(dims, 522)
    b = synth.make_source(dims, 523)
    lat = _lat(dims, U)
    _, dm, _, _, _ = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, 400, force=False)
    vals = [lat.sign_apply_deriv(dev(b[None]), MU, k, x=dev(x[None]), want_vectors=False)[2][0] for k in (300, 400)]
    trunc = abs(vals[1] - vals[0])
    assert trunc < 1e-8 * abs(vals[1])
    assert abs(dm - vals[1]) < 1e-8 * abs(vals[1])


def test_vjp_mixed_precision_bounds():
    """FP32 Lanczos vectors (FP64 scalars and gradient algebra) against the FP64
    gradient at the same k; bounds measured here (4^4, k = 96)."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, print_case, rel
    dims, k = (4, 4, 4, 4), 96
    print_case(test="vjp_mixed", dims=dims, k=k)
    U = synth.make_links(dims, 0.4, 531)
    x = synth.make_source(dims, 532)
    b = synth.make_source(dims, 533)
    out = {}
    for prec in (0, 1):
        lat = ovderiv.Lattice(dims, precision=prec)
        lat.set_links(dev(U))
        out[prec] = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, force=True, wirtinger=False)
    e_s = abs(out[1][0] - out[0][0]) / abs(out[0][0])
    e_d = abs(out[1][1] - out[0][1]) / abs(out[0][1])
    e_f = rel(host(out[1][2]), host(out[0][2]))
    print(f"mixed gradient deviations: s {e_s:.1e}, ds/dmu {e_d:.1e}, force {e_f:.1e}")
    assert e_s < 1e-5 and e_d < 1e-4 and e_f < 1e-4


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [20, 70])
def test_vjp_recomputed_basis_matches_stored(prec, k):
    """The recompute form (left basis only, turned into Z in place; the right
    basis regenerated by a second run and folded into the force 32 vectors at
    a time, here one partial chunk at k = 20 and chunks 32 + 32 + 6 at k = 70)
    against the stored form on a lattice whose volume is not a multiple of 64:
    the regenerated vectors are the same, so s, ds/dmu, the force and the
    Wirtinger derivatives agree to 1e-13; in FP64 the stored form also matches
    the oracle's Krylov gradient to 1e-10."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, print_case, rel
    dims = (5, 3, 4, 3)
    print_case(test="vjp_recompute", dims=dims, k=k, prec=prec)
    U = synth.make_links(dims, 0.5, 541)
    x = synth.make_source(dims, 542)
    b = synth.make_source(dims, 543)
    out = {}
    for rc in (0, 1):
        lat = ovderiv.Lattice(dims, precision=prec, basis_recompute=bool(rc))
        lat.set_links(dev(U))
        out[rc] = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, force=True, wirtinger=True)
        assert lat.last_stats.basis_recomputed == rc
        lat.close()
    (s0, d0, F0, U0, C0), (s1, d1, F1, U1, C1) = out[0], out[1]
    devs = [abs(s1 - s0) / abs(s0), abs(d1 - d0) / abs(d0)] + \
        [rel(host(a), host(c)) for a, c in ((F1, F0), (U1, U0), (C1, C0))]
    print(f"  prec {prec} k {k}: regenerated against stored " + " ".join(f"{e:.1e}" for e in devs), flush=True)
    assert max(devs) < 1e-13
    if prec == 0:
        s_r, dm_r, F_r, _ = vjp.krylov_vjp(U, dims, MU, x, b, k)
        assert abs(s0 - s_r) < 1e-10 * abs(s_r) and abs(d0 - dm_r) < 1e-10 * abs(dm_r)
        assert rel(host(F0), F_r) < 1e-10


def test_vjp_auto_mode_stores_when_memory_allows():
    """Default (auto) mode: a small lattice's gradient fits, so the bases are stored."""
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="vjp_auto", dims=dims)
    U = synth.make_links(dims, 0.5, 551)
    lat = _lat(dims, U)
    x = synth.make_source(dims, 552)
    lat.sign_apply_vjp(dev(x[None]), dev(x[None]), MU, 16)
    assert lat.last_stats.basis_recomputed == 0


def test_u1_current_against_finite_differences_and_oracle():
    """ds/dTheta_nu(y) = i tr F_nu(y), the derivative along the external U(1)
    field of Sec. 4 (dsdtheta output of ovd_sign_apply_vjp): on 2^4 at k = 160
    (converged) against central differences of the oracle's dense
    <x|sgn(H)|b> for the phase of every link; on 4^4 at k = 96 against the
    oracle's Krylov gradient at the same k."""
    from gpu_helpers import dev, host, print_case, rel
    dims = (2, 2, 2, 2)
    print_case(test="vjp_u1", dims=dims, k=160)
    U = synth.make_links(dims, 0.5, 41)
    x = synth.make_source(dims, 42)
    b = synth.make_source(dims, 43)
    lat = _lat(dims, U)
    lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, 160, force=False, u1=True)
    D = host(lat.last_dsdtheta)
    lat.close()
    h = 1e-5

    def s_of(Uv):
        return np.vdot(x.ravel(), matfun.sign_schur(dirac.dense_h(Uv, dims, MU)) @ b.ravel())

    for nu in range(4):
        for site in range(U.shape[1]):
            Up, Um = U.copy(), U.copy()
            Up[nu, site] = np.exp(1j * h) * Up[nu, site]
            Um[nu, site] = np.exp(-1j * h) * Um[nu, site]
            fd = (s_of(Up) - s_of(Um)) / (2 * h)
            assert abs(fd - D[nu, site]) < 1e-8, (nu, site)
    dims, k = (4, 4, 4, 4), 96
    print_case(test="vjp_u1", dims=dims, k=k)
    U = synth.make_links(dims, 0.4, 501)
    x = synth.make_source(dims, 502)
    b = synth.make_source(dims, 503)
    _, _, F_r, _ = vjp.krylov_vjp(U, dims, MU, x, b, k)
    lat = _lat(dims, U)
    lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, force=False, u1=True)
    assert rel(host(lat.last_dsdtheta), vjp.u1_derivative(F_r)) < 1e-10
    lat.close()


def _fcols(v):
    return np.ascontiguousarray(v.T.reshape(v.shape[1], -1, 4, 3))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_vjp_deflated_against_oracle(prec):
    """Gradient of <x|sgn(H)|b> with the 12 eigenpairs of smallest |lambda|
    deflated (oracle eigen-data, rough small-gap 4x2x2x4 field): against the
    oracle's krylov_vjp_deflated at the same k (FP64 to 1e-10; mixed to 2e-3:
    measured 5.6e-4 for ds/dmu on this rough field, where k = 96 is far from
    converged), the stored and regenerated-basis forms identical in FP64, and
    at k = 600 the dense gradient to 1e-9."""
    from paper_1611_00195_amd import ovderiv
    from oracle import deflation
    from gpu_helpers import dev, host, print_case, rel
    dims, k, m = (4, 2, 2, 4), 96, 12
    print_case(test="vjp_deflated", dims=dims, k=k, m=m, prec=prec)
    U = synth.make_links(dims, 1.0, 301)
    x = synth.make_source(dims, 42)
    b = synth.make_source(dims, 43)
    H = dirac.dense_h(U, dims, MU)
    lam, R, L = deflation.eigpairs_dense(H, m)
    s_r, dm_r, F_r, _ = vjp.krylov_vjp_deflated(U, dims, MU, x, b, k, lam, R, L)
    out = {}
    for rc in (False, True):
        lat = ovderiv.Lattice(dims, precision=ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED, basis_recompute=rc)
        lat.set_links(dev(U))
        lat.set_deflation(MU, lam, dev(_fcols(R)), dev(_fcols(L)))
        out[rc] = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, k, force=True, u1=True)
        out[rc] = out[rc] + (host(lat.last_dsdtheta),)
        assert lat.last_stats.basis_recomputed == int(rc)
        lat.close()
    s, dm, F, _, _, D = out[False]
    es, ed, eF = abs(s - s_r) / abs(s_r), abs(dm - dm_r) / abs(dm_r), rel(host(F), F_r)
    eD = rel(D, vjp.u1_derivative(F_r))
    print(f"  {prec} against the oracle: s {es:.2e}, ds/dmu {ed:.2e}, force {eF:.2e}, U(1) {eD:.2e}", flush=True)
    tol = 1e-10 if prec == "fp64" else 2e-3
    assert max(es, ed, eF, eD) < tol
    s2, dm2, F2, _, _, _ = out[True]
    dr = max(abs(s2 - s) / abs(s), abs(dm2 - dm) / abs(dm), rel(host(F2), host(F)))
    print(f"  {prec} regenerated basis against stored: {dr:.2e}", flush=True)
    assert dr < (1e-12 if prec == "fp64" else 1e-6)
    if prec == "fp64":
        s_d, dm_d, F_d = vjp.dense_vjp(U, dims, MU, x, b)
        lat = ovderiv.Lattice(dims)
        lat.set_links(dev(U))
        lat.set_deflation(MU, lam, dev(_fcols(R)), dev(_fcols(L)))
        s6, dm6, F6, _, _ = lat.sign_apply_vjp(dev(x[None]), dev(b[None]), MU, 600)
        lat.close()
        e6 = (abs(s6 - s_d) / abs(s_d), abs(dm6 - dm_d) / abs(dm_d), rel(host(F6), F_d))
        print(f"  k=600 against the dense gradient: {e6}", flush=True)
        assert max(e6) < 1e-9
