"""Uneven batch across lattices (ovd_sign_apply_deriv_batch): every lattice's
result equals its own single call, and the oracle for one source per lattice."""
import numpy as np
import pytest

import synth
from oracle import tsl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1])
def test_uneven_batch_matches_single_calls(prec):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, ops, print_case
    shapes = [((4, 4, 4, 4), 3, 40), ((4, 4, 4, 6), 2, 56), ((6, 4, 2, 4), 4, 32)]
    print_case(test="uneven_batch", shapes=shapes, prec=prec)
    jobs, singles, data = [], [], []
    for i, (dims, nr, k) in enumerate(shapes):
        U = synth.make_links(dims, 0.5, 801 + i)
        lat = ovderiv.Lattice(dims, precision=prec, stream=torch.cuda.Stream())
        lat.set_links(dev(U))
        b = dev(synth.make_sources(dims, nr, 810 + i))
        x = dev(synth.make_sources(dims, nr, 820 + i))
        mus = list(np.linspace(0.1, 0.4, nr))
        jobs.append((lat, b, mus, k, x))
        data.append((U, dims, b, x, mus, k))
    res = ovderiv.sign_apply_deriv_batch(jobs)
    for (lat, b, mus, k, x), r in zip(jobs, res):
        _, _, s1 = lat.sign_apply_deriv(b, mus, k, x=x, want_vectors=False)
        assert r == s1
    if prec == 0:
        from gpu_helpers import host
        for (U, dims, b, x, mus, k), r in zip(data, res):
            h, hd, dh, dhd = ops(U, dims, mus[0])
            d, _, _ = tsl.krylov_sign_deriv(h, hd, dh, dhd, host(b)[0].ravel(), k)
            ref = np.vdot(host(x)[0].ravel(), d)
            assert abs(r[0] - ref) < 1e-10 * abs(ref)


def test_batch_rejects_repeated_handle():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims = (4, 4, 4, 4)
    print_case(test="batch_repeated", dims=dims)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(synth.make_links(dims, 0.5, 830)))
    b = dev(synth.make_sources(dims, 1, 831))
    with pytest.raises(ovderiv.OvdError):
        ovderiv.sign_apply_deriv_batch([(lat, b, 0.3, 8, b), (lat, b, 0.3, 8, b)])
