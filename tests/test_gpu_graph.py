"""Replays of the recorded Lanczos loop (HIP graph) against launches one by one.

The graph holds only kernel launches (no memset nodes).  Each replay is
checked against the eagerly launched result, with the program's own eager
work and synchronisations between replays, across a change of shape and of
the link contents.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pair(dims, U, prec):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev
    g = ovderiv.Lattice(dims, precision=prec, use_graph=True)
    e = ovderiv.Lattice(dims, precision=prec, use_graph=False)
    Ut = dev(U)
    g.set_links(Ut)
    e.set_links(Ut)
    return g, e


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager(prec):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, print_case
    dims, mu = (4, 4, 4, 4), 0.3
    print_case(test="graph_replays", dims=dims, prec=prec)
    U = synth.make_links(dims, 0.5, 601)
    g, e = _pair(dims, U, prec)
    b = dev(synth.make_sources(dims, 3, 602))
    x = dev(synth.make_sources(dims, 3, 603))
    ref = {}
    for k in (24, 40):
        y, dy, s = e.sign_apply_deriv(b, mu, k, x=x)
        ref[k] = (host(y), host(dy), s)
    v = dev(synth.make_sources(dims, 2, 604))
    for rep, k in enumerate((24, 24, 40, 24, 40)):
        y, dy, s = g.sign_apply_deriv(b, mu, k, x=x)
        assert np.array_equal(host(y), ref[k][0]) and np.array_equal(host(dy), ref[k][1]), (rep, k)
        assert s == ref[k][2], (rep, k)
        # eager work of the program between replays
        w = g.apply_op(ovderiv.OP_H, mu, v)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(w)).all()
    # new link contents behind the same handle: replays read them
    U2 = synth.make_links(dims, 0.5, 605)
    g.set_links(dev(U2))
    e.set_links(dev(U2))
    for _ in range(2):
        y2, _, s2 = g.sign_apply_deriv(b, mu, 24, x=x)
        y2e, _, s2e = e.sign_apply_deriv(b, mu, 24, x=x)
        assert np.array_equal(host(y2), host(y2e)) and s2 == s2e
    assert not np.array_equal(host(y2), ref[24][0])


def test_graph_sign_and_vjp_match_eager():
    from gpu_helpers import dev, host, print_case
    dims, mu, k = (4, 2, 2, 4), 0.3, 32
    print_case(test="graph_sign_vjp", dims=dims, k=k)
    U = synth.make_links(dims, 0.5, 611)
    g, e = _pair(dims, U, 0)
    b = dev(synth.make_sources(dims, 2, 612))
    ye = host(e.sign_apply(b, mu, k))
    se = e.sign_apply_vjp(b[:1].contiguous(), b[1:].contiguous(), mu, k)
    for _ in range(3):
        assert np.array_equal(host(g.sign_apply(b, mu, k)), ye)
        sg = g.sign_apply_vjp(b[:1].contiguous(), b[1:].contiguous(), mu, k)
        assert sg[0] == se[0] and sg[1] == se[1]
        assert np.array_equal(host(sg[2]), host(se[2]))
        torch.cuda.synchronize()
