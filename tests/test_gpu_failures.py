"""Failure paths of the library on the GPU: every case returns a status code
(never a silent wrong result) and every kernel exits normally.

  * non-finite links: the recurrence detects the non-finite reductions and
    the call returns OVD_ENAN; the handle works again after good links;
  * x orthogonal to b in the gradient: the bilinear two-sided Lanczos has
    w_1^dag v_1 = 0, a serious breakdown at step 0 (OVD_EBREAKDOWN);
  * degenerate eigenvalues where derivative pairs are asked for (free field,
    lowest shell of 24 made of four six-fold values): OVD_ENOCONV from the
    eigensolver, since the eigenvector derivatives are undefined there;
  * a memory budget smaller than the Krylov basis: the call regenerates the
    basis instead of storing it, with the same result;
  * deflation data that no longer belong to the call: new links remove every
    set; a set built along one link direction refuses another.
"""
import numpy as np
import pytest

import synth
from oracle import deflation, dirac

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_nan_links_return_enan_and_handle_recovers():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="fail_nan", dims=dims)
    U = synth.make_links(dims, 0.5, 801)
    Ubad = U.copy()
    Ubad[3, 17, 1, 2] = np.nan
    b = synth.make_sources(dims, 2, 802)
    x = synth.make_sources(dims, 2, 803)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(Ubad))
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.sign_apply_deriv(dev(b), 0.3, 32, x=dev(x), want_vectors=False)
    assert ei.value.status == ovderiv.OVD_ENAN
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.sign_apply(dev(b), 0.3, 32)
    assert ei.value.status == ovderiv.OVD_ENAN
    lat.set_links(dev(U))
    _, _, s = lat.sign_apply_deriv(dev(b), 0.3, 32, x=dev(x), want_vectors=False)
    assert all(np.isfinite(v) for v in s)
    lat.close()


def test_orthogonal_x_and_b_break_down_at_step_zero():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="fail_orth", dims=dims)
    U = synth.make_links(dims, 0.5, 804)
    b = synth.make_source(dims, 805)
    x = synth.make_source(dims, 806)
    x = x - np.vdot(b.ravel(), x.ravel()) * b          # b has unit norm: x^dag b = 0
    assert abs(np.vdot(x.ravel(), b.ravel())) < 1e-15
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    with pytest.raises(ovderiv.Breakdown):
        lat.sign_apply_vjp(dev(x[None]), dev(b[None]), 0.3, 32)
    # the statistics carry the step of the breakdown
    from paper_1611_00195_amd.ovderiv import _Stats, lib
    import ctypes
    st = _Stats()
    sc = (ctypes.c_double * 2)()
    xd, bd = dev(x[None]), dev(b[None])
    rc = lib().ovd_sign_apply_vjp(lat._h, ctypes.c_double(0.3), 32, ctypes.c_void_p(xd.data_ptr()),
                                  ctypes.c_void_p(bd.data_ptr()), sc, None, None, None, None, None,
                                  ctypes.byref(st))
    assert rc == ovderiv.OVD_EBREAKDOWN and st.breakdown_step == 0
    lat.close()


def test_degenerate_cluster_at_the_derivative_pairs_is_refused():
    """Pure-gauge links: the lowest modulus shell of H(0.3) on 4^4 holds 24
    eigenvalues, four distinct values six times each (momentum degeneracy).
    The m = 20 set cuts the shell; that alone leaves a valid deflation (any
    set of eigenpairs with L^dag R = 1 gives an H-invariant projector), but the
    derivatives of l = 5 pairs cannot be defined: by pigeonhole two of them
    share an eigenvalue, and the formula divides by lam_j - lam_i."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="fail_cluster", dims=dims, m=20, l=5)
    U, _ = synth.gauge_rotated_unit_links(dims, 5)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.compute_deflation(0.3, 20, 5)
    assert ei.value.status == ovderiv.OVD_ENOCONV and "degenerate" in str(ei.value)
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.get_deflation(0.3)
    assert ei.value.status == ovderiv.OVD_ENODEFL
    lat.close()


def test_memory_budget_switches_to_the_regenerated_basis():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case, rel
    dims, k = (4, 4, 4, 6), 60
    print_case(test="fail_budget", dims=dims, k=k)
    U = synth.make_links(dims, 0.5, 807)
    b = synth.make_sources(dims, 2, 808)
    x = synth.make_source(dims, 809)
    out = {}
    for budget in (0, 1 << 20):   # the basis takes 2 * 60 * 2 * 12 * 384 * 16 B = 17.7 MB
        lat = ovderiv.Lattice(dims, mem_budget=budget)
        lat.set_links(dev(U))
        y, dy, _ = lat.sign_apply_deriv(dev(b), 0.3, k)
        rec = lat.last_stats.basis_recomputed
        s, dm, F, _, _ = lat.sign_apply_vjp(dev(x[None]), dev(b[:1]), 0.3, k)
        out[budget] = (y, dy, rec, lat.last_stats.basis_recomputed, s, dm, F)
        lat.close()
    y0, dy0, r0, v0, s0, dm0, F0 = out[0]
    y1, dy1, r1, v1, s1, dm1, F1 = out[1 << 20]
    assert (r0, v0, r1, v1) == (0, 0, 1, 1)
    assert rel(dy1.cpu().numpy(), dy0.cpu().numpy()) < 1e-12
    assert rel(y1.cpu().numpy(), y0.cpu().numpy()) < 1e-12
    assert abs(s1 - s0) <= 1e-13 * abs(s0) and abs(dm1 - dm0) <= 1e-12 * abs(dm0)
    assert rel(F1.cpu().numpy(), F0.cpu().numpy()) < 1e-12


def _f(v):
    return np.ascontiguousarray(v.T.reshape(v.shape[1], -1, 4, 3))


def test_new_links_remove_deflation_sets():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims, mu, k = (4, 2, 2, 4), 0.3, 48
    print_case(test="fail_stale_links", dims=dims)
    U = synth.make_links(dims, 1.0, 301)
    U2 = synth.make_links(dims, 1.0, 302)
    H = dirac.dense_h(U, dims, mu)
    dH = dirac.dense_dh_dmu(U, dims, mu)
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH, 12)
    b = synth.make_sources(dims, 1, 810)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    lat.set_deflation(mu, lam, dev(_f(R)), dev(_f(L)), 6, dev(_f(dR[:, :6])), dev(_f(dL[:, :6])))
    lat.set_links(dev(U2))
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.get_deflation(mu)
    assert ei.value.status == ovderiv.OVD_ENODEFL
    y, dy, _ = lat.sign_apply_deriv(dev(b), mu, k)
    fresh = ovderiv.Lattice(dims)
    fresh.set_links(dev(U2))
    y2, dy2, _ = fresh.sign_apply_deriv(dev(b), mu, k)
    assert torch.equal(dy, dy2) and torch.equal(y, y2)
    lat.close()
    fresh.close()


def test_link_direction_set_refuses_another_direction():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case, rel
    dims, mu, k = (4, 2, 2, 4), 0.3, 48
    print_case(test="fail_stale_dir", dims=dims)
    U = synth.make_links(dims, 1.0, 301)
    dU1 = dirac.link_tangent(synth.make_su3_direction(dims, 311), U)
    dU2 = dirac.link_tangent(synth.make_su3_direction(dims, 312), U)
    H = dirac.dense_h(U, dims, mu)
    dH1 = dirac.dense_dh_dlink(dU1, dims, mu)
    lam, R, L, dlam, dR, dL = deflation.eig_derivs_dense(H, dH1, 8)
    b = synth.make_sources(dims, 1, 811)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    # a link-direction set needs its direction
    with pytest.raises(ovderiv.OvdError):
        lat.set_deflation(mu, lam, dev(_f(R)), dev(_f(L)), 4, dev(_f(dR[:, :4])), dev(_f(dL[:, :4])),
                          direction="link", dU=None)
    lat.set_deflation(mu, lam, dev(_f(R)), dev(_f(L)), 4, dev(_f(dR[:, :4])), dev(_f(dL[:, :4])),
                      direction="link", dU=dev(dU1))
    _, dy1, _ = lat.sign_apply_deriv(dev(b), mu, k, direction="link", dU=dev(dU1))
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.sign_apply_deriv(dev(b), mu, k, direction="link", dU=dev(dU2))
    assert ei.value.status == ovderiv.OVD_EINVAL
    with pytest.raises(ovderiv.OvdError) as ei:
        lat.sign_apply_deriv(dev(b), mu, k)
    assert ei.value.status == ovderiv.OVD_EINVAL
    # the same direction passed again (a fresh copy of the same values) is accepted
    _, dy1b, _ = lat.sign_apply_deriv(dev(b), mu, k, direction="link", dU=dev(dU1.copy()))
    assert rel(dy1b.cpu().numpy(), dy1.cpu().numpy()) == 0.0
    lat.close()
