"""Every launch shape of the stencils (XCD work order x site groups per block x
paired or sequential form x one or two right-hand sides per thread of Dw.v),
forced through the options, against the oracle; and the autotuner's choice."""
import pytest

import synth
from oracle import tsl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape", [(0, 1), (0, 2), (1, 1), (1, 2), (0, 4), (1, 4), (0, 8), (1, 8),
                                   (0, 1, 1), (0, 2, 1), (1, 1, 1), (1, 2, 1), (0, 4, 1), (1, 4, 1), (1, 8, 1),
                                   (0, 4, 0, 2), (1, 2, 0, 2)])
def test_forced_shapes_deriv_and_sign(shape):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, ops, print_case, rel
    # xy-plane of 12 x 11 = 132 sites: the plane-in-LDS shape (8) applies
    dims, k, nrhs, mu = ((12, 11, 2, 4) if shape[1] == 8 else (4, 4, 4, 4)), 32, 8, 0.3
    print_case(test="shapes", shape=shape, dims=dims, nrhs=nrhs)
    U = synth.make_links(dims, 0.5, 901)
    lat = ovderiv.Lattice(dims, shape=shape)
    lat.set_links(dev(U))
    b = synth.make_sources(dims, nrhs, 902)
    h, hd, dh, dhd = ops(U, dims, mu)
    if shape[1] in (1, 2, 8):       # derivative stencil shapes
        y, dy, _ = lat.sign_apply_deriv(dev(b), mu, k)
        for r in (0, nrhs - 1):
            dref, yref, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, b[r].ravel(), k)
            assert rel(host(dy)[r], dref) < 1e-10 and rel(host(y)[r], yref) < 1e-10
    if shape[1] in (2, 4, 8):       # plain stencil shapes (sign, Dw.v)
        y = host(lat.sign_apply(dev(b), mu, k))
        for r in (0, nrhs - 1):
            ref, _ = tsl.krylov_sign(h, hd, b[r].ravel(), b[r].ravel(), k)
            assert rel(y[r], ref) < 1e-10
        from oracle import dirac
        out = host(lat.apply_op(ovderiv.OP_H, mu, dev(b)))   # Dw.v: shape 8 falls back to 4
        for r in (0, nrhs - 1):
            assert rel(out[r], dirac.flat(dirac.apply_h(U, b[r].ravel(), dims, mu))) < 1e-14


@pytest.mark.parametrize("shape", [(1, 1, 2), (1, 2, 2), (0, 2, 2)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_form_of_the_plain_pair(shape, prec):
    """The split form of the plain pair (H vhat and H^dag what of a site in two
    waves), forced, against the oracle on a lattice whose volume is not a
    multiple of the 64-site group: sgn(H)b for three sources (FP64 to 1e-10,
    mixed to 5e-5 as the paired form) and, in FP64, the gradient's bilinear
    run (s, ds/dmu and the force to 1e-10).  The split form computes each
    output as the sequential form does; with 2 groups per block (the same
    blocks and partial sums) it matches that form bit for bit."""
    import numpy as np

    from paper_1611_00195_amd import ovderiv
    from oracle import vjp
    from gpu_helpers import dev, host, ops, print_case, rel
    # XCD order 0 needs a multiple of 8 sources
    dims, k, nrhs, mu = (5, 3, 4, 3), 24, (8 if shape[0] == 0 else 3), 0.25
    print_case(test="split_form", shape=shape, prec=prec, dims=dims, nrhs=nrhs)
    p = ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED
    U = synth.make_links(dims, 0.5, 911)
    b = synth.make_sources(dims, nrhs, 912)
    x = synth.make_source(dims, 913)
    h, hd, _, _ = ops(U, dims, mu)
    lat = ovderiv.Lattice(dims, precision=p, shape=shape)
    lat.set_links(dev(U))
    y = host(lat.sign_apply(dev(b), mu, k))
    assert f"map{shape[0]},gpb{shape[1]},split" in lat.tuned_shapes()
    tol = 1e-10 if prec == "fp64" else 5e-5
    for r in sorted({0, 1, nrhs - 1}):
        ref, _ = tsl.krylov_sign(h, hd, b[r].ravel(), b[r].ravel(), k)
        assert rel(y[r], ref) < tol
    if shape[1] == 2:   # the same blocks and partial sums as the sequential form
        seq = ovderiv.Lattice(dims, precision=p, shape=(shape[0], 2, 1))
        seq.set_links(dev(U))
        assert np.array_equal(host(seq.sign_apply(dev(b), mu, k)), y)
        seq.close()
    if prec == "fp64":
        s, dm, F = lat.sign_apply_vjp(dev(x[None]), dev(b[:1]), mu, k, force=True)[:3]
        s_r, dm_r, F_r, _ = vjp.krylov_vjp(U, dims, mu, x, b[0], k)
        assert abs(s - s_r) < 1e-10 * abs(s_r) and abs(dm - dm_r) < 1e-10 * abs(dm_r)
        assert rel(host(F), F_r) < 1e-10
    lat.close()


def test_autotuner_records_a_shape():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="autotune", dims=dims)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(synth.make_links(dims, 0.5, 903)))
    b = dev(synth.make_sources(dims, 8, 904))
    lat.sign_apply_deriv(b, 0.3, 8, x=b, want_vectors=False)
    lat.apply_op(ovderiv.OP_H, 0.3, b)
    shapes = lat.tuned_shapes()
    assert "tsl:d:1:8=" in shapes and "op:d:0:8=" in shapes


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sequential_and_paired_forms_against_oracle(prec):
    """Both forms of the stencil (paired and sequential) against the oracle on
    a lattice whose volume is not a multiple of the 64-site group, with the
    x-projection of the scalar mode: FP64 to 1e-10; mixed precision to 5e-5
    (sign) and 3e-4 (derivative, vectors and <x|dy>), about three times the
    measured 1.8e-5 and 9.0e-5 of this short (k = 24) recurrence on MI355X.
    The two forms round differently where the mu-derivative terms enter, so
    they are compared with the oracle, not bit for bit with each other."""
    import numpy as np

    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, ops, print_case, rel
    dims, k, nrhs, mu = (5, 3, 4, 3), 24, 3, 0.25
    print_case(test="seq_and_paired", prec=prec, dims=dims, nrhs=nrhs)
    p = ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED
    Uh = synth.make_links(dims, 0.5, 905)
    bh = synth.make_sources(dims, nrhs, 906)
    xh = synth.make_sources(dims, nrhs, 907)
    h, hd, dh, dhd = ops(Uh, dims, mu)
    refs = []
    for r in range(nrhs):
        dref, yref, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, bh[r].ravel(), k)
        sref, _ = tsl.krylov_sign(h, hd, bh[r].ravel(), bh[r].ravel(), k)
        refs.append((yref, dref, np.vdot(xh[r].ravel(), dref), sref))
    t_sign, t_der = (1e-10, 1e-10) if prec == "fp64" else (5e-5, 3e-4)
    U, b, x = dev(Uh), dev(bh), dev(xh)
    for seq in (0, 1):
        lat = ovderiv.Lattice(dims, precision=p, shape=(1, 2, seq))
        lat.set_links(U)
        y, dy, s = lat.sign_apply_deriv(b, mu, k, x=x)
        ys = host(lat.sign_apply(b, mu, k))
        assert ("seq" in lat.tuned_shapes()) == bool(seq)
        lat.close()
        y, dy = host(y), host(dy)
        e_sign = e_der = 0.0
        for r in range(nrhs):
            yref, dref, sref_x, sref = refs[r]
            e_sign = max(e_sign, rel(y[r], yref), rel(ys[r], sref))
            e_der = max(e_der, rel(dy[r], dref),
                        abs(complex(s[r]) - sref_x) / (np.linalg.norm(xh[r]) * np.linalg.norm(dref)))
        print(f"{prec} seq={seq}: sign {e_sign:.2e}  derivative {e_der:.2e}")
        assert e_sign < t_sign and e_der < t_der


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [6, 5])
def test_dwv_two_rhs_per_thread(prec, nrhs):
    """Dw.v with two right-hand sides per thread (forced) against the oracle's
    H and Dw, on a ragged lattice: 6 sources (3 pairs, the contiguous XCD order)
    and 5 (odd: one per thread).  FP64 to 1e-14, FP32 to 1e-6."""
    from paper_1611_00195_amd import ovderiv
    from oracle import dirac
    from gpu_helpers import dev, host, print_case, rel
    dims, mu = (5, 3, 4, 3), 0.35
    print_case(test="dwv_rp2", prec=prec, nrhs=nrhs, dims=dims)
    U = synth.make_links(dims, 0.5, 911)
    b = synth.make_sources(dims, nrhs, 912)
    lat = ovderiv.Lattice(dims, precision=ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED, shape=(0, 4, 0, 2))
    lat.set_links(dev(U))
    tol = 1e-14 if prec == "fp64" else 1e-6
    for op, ref in ((ovderiv.OP_H, dirac.apply_h), (ovderiv.OP_DW, dirac.apply_dw)):
        out = host(lat.apply_op(op, mu, dev(b)))
        for r in range(nrhs):
            assert rel(out[r], dirac.flat(ref(U, b[r].ravel(), dims, mu))) < tol, (op, r)
    assert ("rp2" in lat.tuned_shapes()) == (nrhs % 2 == 0)
    lat.close()


@pytest.mark.parametrize("nseg", [1, 2, 4])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_time_marching_form(prec, order, nseg):
    """The time-marching form of the d/dmu stencil, forced (XCD order, 1, 2 or
    4 time segments), against the oracle on a 12 x 11 x 3 x 5 lattice.  Its 5
    time slices split into segments of 5, of 3 + 2, and of 2 + 2 + 1 with an
    empty fourth; the first slice of each segment takes its backward time hop
    from the slice before (across the time boundary for the first segment),
    and the last slice its forward hop across the boundary.  sgn(H)b, d/dmu
    sgn(H)b and <x|dy> for the first and last of 8 sources: FP64 to 1e-10,
    mixed to 3e-4 (the bound of the paired and sequential forms).  In FP64 the
    result also agrees with the plane-in-LDS shape to 1e-11 (the two sum the
    hops and the partial sums in different orders).  The seeds give a field
    on which the oracle's own result moves by at most 6e-14 under
    rounding-level noise (with links of seed 921 the last source moves by
    3.8e-10, and no two FP64 summation orders agree to 1e-10 there)."""
    import numpy as np

    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, ops, print_case, rel
    dims, k, nrhs, mu = (12, 11, 3, 5), 32, 8, 0.3
    print_case(test="time_marching", prec=prec, order=order, nseg=nseg, dims=dims, nrhs=nrhs)
    p = ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED
    Uh = synth.make_links(dims, 0.5, 931)
    bh = synth.make_sources(dims, nrhs, 932)
    xh = synth.make_sources(dims, nrhs, 933)
    U, b, x = dev(Uh), dev(bh), dev(xh)
    lat = ovderiv.Lattice(dims, precision=p, shape=(order, nseg, 3))
    lat.set_links(U)
    y, dy, s = lat.sign_apply_deriv(b, mu, k, x=x)
    assert f"map{order},gpb{nseg},march" in lat.tuned_shapes()
    lat.close()
    y, dy = host(y), host(dy)
    h, hd, dh, dhd = ops(Uh, dims, mu)
    tol = 1e-10 if prec == "fp64" else 3e-4
    err = 0.0
    for r in (0, nrhs - 1):
        dref, yref, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, bh[r].ravel(), k)
        sx = np.vdot(xh[r].ravel(), dref)
        err = max(err, rel(y[r], yref), rel(dy[r], dref),
                  abs(complex(s[r]) - sx) / (np.linalg.norm(xh[r]) * np.linalg.norm(dref)))
    print(f"{prec} order {order}, {nseg} segments: {err:.2e} from the oracle")
    assert err < tol
    if prec == "fp64":
        pl = ovderiv.Lattice(dims, precision=p, shape=(order, 8))
        pl.set_links(U)
        yp, dyp, sp = pl.sign_apply_deriv(b, mu, k, x=x)
        pl.close()
        d = max(rel(y, host(yp)), rel(dy, host(dyp)))
        print(f"  from the plane shape: {d:.2e}")
        assert d < 1e-11


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dwv_plane_in_lds(prec, order):
    """Dw.v with two right-hand sides per thread and the xy-plane in LDS
    (forced; a 12 x 11 x 3 x 5 lattice, 16 sources: 8 pairs, so both XCD
    orders apply) against the oracle's H and Dw (FP64 to 1e-14, FP32 to 1e-6),
    and against the paired form without LDS, which applies the same hops with
    the same arithmetic up to the compiler's choice of fused multiply-adds
    (to 1e-15 in FP64 and 4e-7 in FP32, relative to the largest element; at
    14^4 the two differ by 3.0e-16 and 1.5e-7)."""
    import numpy as np

    from paper_1611_00195_amd import ovderiv
    from oracle import dirac
    from gpu_helpers import dev, host, print_case, rel
    dims, mu, nrhs = (12, 11, 3, 5), 0.35, 16
    print_case(test="dwv_plane", prec=prec, order=order, nrhs=nrhs, dims=dims)
    p = ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED
    U = synth.make_links(dims, 0.5, 941)
    b = synth.make_sources(dims, nrhs, 942)
    lat = ovderiv.Lattice(dims, precision=p, shape=(order, 8, 0, 2))
    lat.set_links(dev(U))
    pair = ovderiv.Lattice(dims, precision=p, shape=(order, 4, 0, 2))
    pair.set_links(dev(U))
    tol, tpair = (1e-14, 1e-15) if prec == "fp64" else (1e-6, 4e-7)
    for op, ref in ((ovderiv.OP_H, dirac.apply_h), (ovderiv.OP_DW, dirac.apply_dw)):
        out = host(lat.apply_op(op, mu, dev(b)))
        outp = host(pair.apply_op(op, mu, dev(b)))
        d = np.abs(out - outp).max() / np.abs(outp).max()
        print(f"{prec} order {order} op {op}: {d:.2e} from the paired form")
        assert d < tpair
        for r in (0, 7, nrhs - 1):
            assert rel(out[r], dirac.flat(ref(U, b[r].ravel(), dims, mu))) < tol, (op, r)
    assert f"map{order},gpb8,rp2" in lat.tuned_shapes()
    lat.close()
    pair.close()
