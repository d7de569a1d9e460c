"""GPU parity against stored oracle references at the workloads' full sizes
and Krylov dimensions.

The references in tests/golden/*.json are written by tests/golden/make_golden.py,
which calls only the CPU oracle (oracle/) and the input generators (synth/);
the oracle needs minutes to hours per case at these sizes.  Each case stores
<x|dy>, <x|y>, the norms of y = sgn(H) b and dy = d/dt sgn(H) b, both vectors
at 64 seeded sites (all 12 components), and every Lanczos coefficient.

  * 14 x 14^3, k = 400, mu = 0.3 (the headline; Sec. 2 eq. 7): sources 0 and 7
    of the benchmark's 8-source storage-free launch, FP64 to 1e-10 and mixed
    precision to 1e-5; the vectors y, dy element by element at the sampled
    sites; the plain sgn(H) b; the drift of alpha, beta, delta over the 400
    steps; the generalised deflation with the GPU's own m = 40 / l = 6 set
    (Sec. 3 eq. 11) within the truncation error of the undeflated reference;
  * 8^4, k = 200, mu in {0, 0.2, 0.4}, the mu and an su(3) link direction;
  * 12^4, k = 300, sources 0 and 63 of the 64-source batch (16 sources x 4 mu),
    undeflated and with the per-mu m = 32 deflation sets computed on the GPU;
  * the uneven batch (its Lanczos steps shared by the four lattices): 6^4 at
    k = 150, 10^4 at k = 250 (both sources), 16^4 at k = 400 and 20 x 20^3 at
    k = 500;
  * the gradient of <x|sgn(H)|b> at 14 x 14^3, k = 400 (source 0 of the
    benchmark): s, ds/dmu, the force at 64 sampled links and the U(1)
    derivative i tr F there, FP64 with the basis stored or regenerated, and
    mixed precision.
"""
import functools
import json
import os

import numpy as np
import pytest

import synth
from oracle import dirac

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@functools.lru_cache(maxsize=None)
def _g(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"reference {name} not generated (python tests/golden/make_golden.py {name})")
    with open(path) as f:
        d = json.load(f)
    return d


def _c(a):
    a = np.asarray(a, dtype=float)
    return a[..., 0] + 1j * a[..., 1]


def _inputs(p):
    dims = tuple(p["dims"])
    U = synth.make_links(dims, p["eps"], p["link_seed"])
    dU = None
    if p["direction"] == "link":
        dU = dirac.link_tangent(synth.make_su3_direction(dims, p["dir_seed"]), U)
    return dims, U, dU


def _site_err(field, g, key):
    """max over the sampled sites and components of |gpu - ref|, relative to
    the largest reference element there"""
    from gpu_helpers import host
    V = int(np.prod(g["params"]["dims"]))
    a = host(field).reshape(V, 12)[np.array(g["sites"])]
    ref = _c(g[key])
    return np.abs(a - ref).max() / np.abs(ref).max()


def _coef_drift(lat, g, rhs, k, block=None):
    """largest relative deviation of alpha, beta, delta from the reference, over
    steps [0, j) for j = 50, 100, ..., k (entry 0 of beta and delta excluded)"""
    a, b, d = (np.array(v) for v in lat.get_tridiag(k, rhs=rhs))
    src = g if block is None else g[block]
    ra, rb, rd = _c(src["alpha"]), _c(src["beta"]), _c(src["delta"])
    dev_a = np.abs(a - ra) / np.abs(ra)
    dev_b = np.abs(b[1:] - rb[1:]) / np.abs(rb[1:])
    dev_d = np.abs(d[1:] - rd[1:]) / np.abs(rd[1:])
    out = {}
    for j in list(range(50, k, 50)) + [k]:
        out[j] = float(max(dev_a[:j].max(), dev_b[:j - 1].max() if j > 1 else 0.0,
                           dev_d[:j - 1].max() if j > 1 else 0.0))
    return out


def _rel(a, b):
    return abs(a - b) / abs(b)


# Bounds of the mixed-precision results (FP32 vectors and stencil, FP64
# scalars) against the FP64 oracle, per workload: about three times the
# largest value measured on MI355X, never above the 1e-5 target where the
# measurement allows it.  Measured, over the launch shapes the tuner has kept
# (each rounds differently): 14 x 14^3 k = 400: <x|dy> up to 2.3e-6, dy at the
# sampled sites up to 4.0e-6, deflated up to 5.2e-6; 8^4 k = 200: 3.5e-6 (dy at
# sites, mu = 0.4); 12^4 k = 300: up to 1.7e-5 (source 63, mu = 0.4; below
# 7e-7 at mu = 0.1); uneven batch: up to 1.1e-6 (the 6^4 run is bounded by
# the oracle's own noise sensitivity instead).
MIXED_TOL = {"c4": 1e-5, "c2": 1e-5, "c3": 5e-5, "c5": 4e-6}


# --------------------------------------------------------------------------
# 14 x 14^3, k = 400, mu = 0.3
# --------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def _c4_fields():
    g0 = _g("c4_r0")
    dims, U, _ = _inputs(g0["params"])
    b = synth.make_sources(dims, 8, 4000)
    x = synth.make_sources(dims, 8, 5000)
    return dims, U, b, x


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_headline_scalar_bench_launch(prec):
    """The benchmark's launch: 8 sources, storage-free scalar mode, autotuned
    shape, graph replay; <x|dy> of sources 0 and 7 against the reference, and
    the coefficient drift of source 0 over the 400 steps."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims, U, b, x = _c4_fields()
    k = 400
    print_case(test="golden_c4_scalar", prec=prec, dims=dims, nrhs=8, k=k)
    lat = ovderiv.Lattice(dims, precision=ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED)
    lat.set_links(dev(U))
    _, _, s = lat.sign_apply_deriv(dev(b), [0.3] * 8, k, x=dev(x), want_vectors=False)
    drift = {r: _coef_drift(lat, _g(f"c4_r{r}"), r, k) for r in (0, 7)}
    lat.close()
    tol = 1e-10 if prec == "fp64" else MIXED_TOL["c4"]
    for r in (0, 7):
        g = _g(f"c4_r{r}")
        ref = complex(*g["xdy"])
        e = _rel(s[r], ref)
        print(f"  source {r}: <x|dy> rel err {e:.2e}; coefficient drift by step {drift[r]}", flush=True)
        assert e <= tol, (r, s[r], ref)
        if prec == "fp64":
            assert drift[r][k] < 1e-8, drift[r]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_headline_vectors(prec):
    """sgn(H) b and d/dmu sgn(H) b as vectors (sources 0 and 7, stored basis):
    element by element at the sampled sites and in norm; the plain sgn(H) b of
    ovd_sign_apply too."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims, U, b, x = _c4_fields()
    k = 400
    src = np.ascontiguousarray(b[[0, 7]])
    print_case(test="golden_c4_vectors", prec=prec, dims=dims, nrhs=2, k=k)
    lat = ovderiv.Lattice(dims, precision=ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED)
    lat.set_links(dev(U))
    y, dy, _ = lat.sign_apply_deriv(dev(src), 0.3, k)
    ys = lat.sign_apply(dev(src), 0.3, k)
    drift = {i: _coef_drift(lat, _g(f"c4_r{r}"), i, k, block="plain") for i, r in enumerate((0, 7))}
    lat.close()
    tol = 1e-10 if prec == "fp64" else MIXED_TOL["c4"]
    for i, r in enumerate((0, 7)):
        g = _g(f"c4_r{r}")
        e = {"dy_sites": _site_err(dy[i], g, "dy_sites"), "y_sites": _site_err(y[i], g, "y_sites"),
             "dy_norm": _rel(float(torch.linalg.vector_norm(dy[i])), g["dy_norm"]),
             "y_norm": _rel(float(torch.linalg.vector_norm(y[i])), g["y_norm"]),
             "plain_sites": _site_err(ys[i], g["plain"] | {"params": g["params"], "sites": g["sites"]}, "y_sites"),
             "plain_norm": _rel(float(torch.linalg.vector_norm(ys[i])), g["plain"]["y_norm"])}
        print(f"  source {r} ({prec}): " + ", ".join(f"{a} {v:.2e}" for a, v in e.items()), flush=True)
        print(f"  source {r}: plain-run coefficient drift by step {drift[i]}", flush=True)
        for key, v in e.items():
            assert v <= tol, (r, key, v)


def test_headline_deflated_within_truncation():
    """The headline workload with its deflation: the m = 40 eigenpairs of
    smallest |lambda| computed on the GPU, the first 6 with derivatives
    (Sec. 3, eq. 8 and 11; the paper's counts at this size).  Deflated and
    undeflated k = 400 results approximate the same sgn(H) b and its
    derivative; they differ by the truncation error of either, which the
    undeflated run puts at the 1e-9 level here (eps_B of Sec. 4 at k = 400).
    FP64 within 1e-7 of the undeflated reference, mixed within 1e-5."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    dims, U, b, x = _c4_fields()
    k = 400
    print_case(test="golden_c4_deflated", dims=dims, m=40, l=6, k=k)
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    lam, st = lat.compute_deflation(0.3, 40, 6)
    print(f"  eigensolver: {st}", flush=True)
    assert st["max_res_right"] <= 1e-10 and st["max_res_left"] <= 1e-10
    _, _, s = lat.sign_apply_deriv(dev(b), [0.3] * 8, k, x=dev(x), want_vectors=False)
    lamd, R, L, dR, dL = lat.get_deflation(0.3)
    lat.close()
    latm = ovderiv.Lattice(dims, precision=ovderiv.MIXED)
    latm.set_links(dev(U))
    latm.set_deflation(0.3, lamd, R, L, 6, dR, dL)
    _, _, sm = latm.sign_apply_deriv(dev(b), [0.3] * 8, k, x=dev(x), want_vectors=False)
    latm.close()
    for r in (0, 7):
        ref = complex(*_g(f"c4_r{r}")["xdy"])
        e64, e32 = _rel(s[r], ref), _rel(sm[r], ref)
        print(f"  source {r}: deflated FP64 vs undeflated reference {e64:.2e}, mixed {e32:.2e}", flush=True)
        assert e64 <= 1e-7 and e32 <= MIXED_TOL["c4"]


# --------------------------------------------------------------------------
# 8^4, k = 200: mu in {0, 0.2, 0.4}, mu and su(3) link directions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("direction", ["mu", "link"])
@pytest.mark.parametrize("mu", [0.0, 0.2, 0.4])
def test_c2_full_k(mu, direction):
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    g = _g(f"c2_mu{mu:.1f}_{direction}")
    p = g["params"]
    dims, U, dU = _inputs(p)
    k = p["k"]
    b = synth.make_source(dims, p["b_seed"])[None]
    x = synth.make_source(dims, p["x_seed"])[None]
    print_case(test="golden_c2", dims=dims, mu=mu, direction=direction, k=k)
    res = {}
    for prec in (ovderiv.FP64, ovderiv.MIXED):
        lat = ovderiv.Lattice(dims, precision=prec)
        lat.set_links(dev(U))
        kw = {} if dU is None else dict(direction="link", dU=dev(dU))
        y, dy, s = lat.sign_apply_deriv(dev(b), mu, k, x=dev(x), **kw)
        drift = _coef_drift(lat, g, 0, k)
        res[prec] = (y, dy, s, drift)
        lat.close()
    ref = complex(*g["xdy"])
    for prec, tol in ((ovderiv.FP64, 1e-10), (ovderiv.MIXED, MIXED_TOL["c2"])):
        y, dy, s, drift = res[prec]
        e = {"xdy": _rel(s[0], ref), "dy_sites": _site_err(dy[0], g, "dy_sites"),
             "y_sites": _site_err(y[0], g, "y_sites"),
             "dy_norm": _rel(float(torch.linalg.vector_norm(dy[0])), g["dy_norm"])}
        print(f"  prec {prec}: " + ", ".join(f"{a} {v:.2e}" for a, v in e.items()) + f"; drift {drift}", flush=True)
        for key, v in e.items():
            assert v <= tol, (prec, key, v)


# --------------------------------------------------------------------------
# 12^4, k = 300: sources 0 and 63 of the 64-source batch
# --------------------------------------------------------------------------
def test_c3_batch_full_k():
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    g0, g63 = _g("c3_r0"), _g("c3_r63")
    dims, U, _ = _inputs(g0["params"])
    k, ns = 300, 16
    print_case(test="golden_c3", dims=dims, nrhs=64, k=k)
    src = synth.make_sources(dims, ns, 1700)
    xs = synth.make_sources(dims, ns, 1800)
    mus = [m for m in (0.1, 0.2, 0.3, 0.4) for _ in range(ns)]
    b = np.concatenate([src] * 4)
    x = np.concatenate([xs] * 4)
    for prec, tol in ((ovderiv.FP64, 1e-10), (ovderiv.MIXED, MIXED_TOL["c3"])):
        lat = ovderiv.Lattice(dims, precision=prec)
        lat.set_links(dev(U))
        _, _, s = lat.sign_apply_deriv(dev(b), mus, k, x=dev(x), want_vectors=False)
        drift = {r: _coef_drift(lat, g, r, k) for r, g in ((0, g0), (63, g63))}
        lat.close()
        for r, g in ((0, g0), (63, g63)):
            e = _rel(s[r], complex(*g["xdy"]))
            print(f"  prec {prec} rhs {r}: <x|dy> {e:.2e}; drift {drift[r]}", flush=True)
            assert e <= tol, (prec, r, e)


def test_c3_deflated_per_mu_within_truncation():
    """The 64-source batch with its per-mu deflation: for each of the four mu
    values the m = 32 eigenpairs of smallest |lambda| computed on the GPU, the
    first 4 with derivatives (Sec. 3, eq. 8 and 11), installed side by side on
    one handle; the call groups its right-hand sides by mu and deflates each
    group with its own set.  Sources 0 (mu = 0.1) and 63 (mu = 0.4) against the
    undeflated oracle references: the two k = 300 approximations differ by
    their truncation errors.  The reference's truncation scale is measured as
    its distance to an undeflated k = 450 run (measured on MI355X: 8.7e-11 at
    mu = 0.1, 3.4e-6 at mu = 0.4, where k = 450 itself has not converged and
    deflation with these 32 pairs barely helps: the 32 |lambda| span only
    2 % at mu = 0.4, 6 % at mu = 0.1); the deflated FP64 result lies within three times that
    (plus 1e-9) of the reference (measured 1.2e-10 and 1.0e-6); mixed within
    5e-5 (measured 3.3e-7 and 5.7e-6)."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    g0, g63 = _g("c3_r0"), _g("c3_r63")
    dims, U, _ = _inputs(g0["params"])
    k, ns, m, l = 300, 16, 32, 4
    print_case(test="golden_c3_deflated", dims=dims, nrhs=64, k=k, m=m, l=l)
    src = synth.make_sources(dims, ns, 1700)
    xs = synth.make_sources(dims, ns, 1800)
    mu_list = (0.1, 0.2, 0.3, 0.4)
    mus = [mu for mu in mu_list for _ in range(ns)]
    b, x = dev(np.concatenate([src] * 4)), dev(np.concatenate([xs] * 4))
    lat = ovderiv.Lattice(dims)
    lat.set_links(dev(U))
    sets = {}
    for mu in mu_list:
        lam, st = lat.compute_deflation(mu, m, l)
        print(f"  mu {mu}: |lambda| {abs(lam[0]):.4f}..{abs(lam[-1]):.4f}, residuals "
              f"{st['max_res_right']:.1e}/{st['max_res_left']:.1e}", flush=True)
        assert st["max_res_right"] <= 1e-10 and st["max_res_left"] <= 1e-10
        sets[mu] = lat.get_deflation(mu)
    _, _, s = lat.sign_apply_deriv(b, mus, k, x=x, want_vectors=False)
    lat.close()
    lat_long = ovderiv.Lattice(dims)        # undeflated, k = 450
    lat_long.set_links(dev(U))
    _, _, s_long = lat_long.sign_apply_deriv(b, mus, 450, x=x, want_vectors=False)
    lat_long.close()
    latm = ovderiv.Lattice(dims, precision=ovderiv.MIXED)
    latm.set_links(dev(U))
    for mu, (lam, R, L, dR, dL) in sets.items():
        latm.set_deflation(mu, lam, R, L, l, dR, dL)
    _, _, sm = latm.sign_apply_deriv(b, mus, k, x=x, want_vectors=False)
    latm.close()
    for r, g in ((0, g0), (63, g63)):
        ref = complex(*g["xdy"])
        e64, e32 = _rel(s[r], ref), _rel(sm[r], ref)
        trunc = _rel(ref, s_long[r])
        e_long = _rel(s[r], s_long[r])
        print(f"  rhs {r}: deflated FP64 vs undeflated reference {e64:.2e}, mixed {e32:.2e}; reference vs "
              f"k = 450 {trunc:.2e}, deflated vs k = 450 {e_long:.2e}", flush=True)
        assert e64 <= 3 * trunc + 1e-9 and e32 <= 5e-5, (r, e64, e32, trunc)


# --------------------------------------------------------------------------
# uneven batch: every lattice inside the four-lattice launch
# --------------------------------------------------------------------------
def test_c5_uneven_batch_full_k():
    """The four lattices of the uneven batch in one shared-step call, FP64 and
    mixed, against the oracle on every lattice: 1e-10 and 4e-6, or ten times
    the oracle's own noise sensitivity where a short run leaves the result
    that loosely determined (6^4 at k = 150: 3.9e-11 at FP64-level noise,
    1.0e-3 at FP32-level noise; the mixed 6^4 result, measured 3.7e-4 off,
    is of that size)."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, print_case
    sizes = [((6, 6, 6, 6), 150), ((10, 10, 10, 10), 250), ((16, 16, 16, 16), 400), ((20, 20, 20, 20), 500)]
    rng = np.random.default_rng(1616)
    print_case(test="golden_c5", sizes=[d for d, _ in sizes])
    for prec, tol in ((ovderiv.FP64, 1e-10), (ovderiv.MIXED, MIXED_TOL["c5"])):
        rng = np.random.default_rng(1616)
        jobs, lats = [], []
        for i, (dims, k) in enumerate(sizes):
            U = synth.make_links(dims, 0.4, 1620 + i)
            b = synth.make_sources(dims, 2, 1630 + 10 * i)
            x = synth.make_sources(dims, 2, 1680 + 10 * i)
            mus = list(rng.uniform(0.0, 0.5, 2))
            lat = ovderiv.Lattice(dims, precision=prec, stream=torch.cuda.Stream())
            lat.set_links(dev(U))
            lats.append(lat)
            jobs.append((lat, dev(b), mus, k, dev(x)))
        res = ovderiv.sign_apply_deriv_batch(jobs)
        torch.cuda.synchronize()
        for lat in lats:
            lat.close()
        for name, li, r in (("c5_6_r0", 0, 0), ("c5_10_r0", 1, 0), ("c5_10_r1", 1, 1), ("c5_16_r0", 2, 0),
                            ("c5_20_r0", 3, 0)):
            path = os.path.join(GOLDEN, f"{name}.json")
            if not os.path.exists(path):
                continue
            g = _g(name)
            assert abs(g["params"]["mu"] - jobs[li][2][r]) < 1e-15
            e = _rel(res[li][r], complex(*g["xdy"]))
            # an unconverged short run (6^4 at k = 150) is determined by the
            # arithmetic only to the oracle's own noise sensitivity (FP64:
            # noise 1e-16, mixed: 1e-7 per operator application); the bound
            # is ten times that where it exceeds the fixed one
            sens = g.get("sensitivity", {}).get("1e-16" if prec == ovderiv.FP64 else "1e-07", 0.0)
            bound = max(tol, 10 * sens)
            print(f"  prec {prec} {name}: <x|dy> {e:.2e} (bound {bound:.1e})", flush=True)
            assert e <= bound, (prec, name, e, bound)


# --------------------------------------------------------------------------
# the gradient at 14 x 14^3, k = 400, mu = 0.3
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,recompute", [("fp64", False), ("fp64", True), ("mixed", False)])
def test_headline_gradient(prec, recompute):
    """ovd_sign_apply_vjp against the oracle's Krylov gradient at the headline
    size: s and ds/dmu relative, the force F and ds/dTheta = i tr F at the
    sampled links relative to the largest |F| entry, FP64 to 1e-10 (with the
    right basis stored or regenerated), mixed precision to 1e-5; the drift of
    the bilinear run's coefficients in FP64."""
    from paper_1611_00195_amd import ovderiv
    from gpu_helpers import dev, host, print_case
    g = _g("c4_vjp")
    p = g["params"]
    dims, U, _ = _inputs(p)
    k, mu = p["k"], p["mu"]
    b = synth.make_source(dims, p["b_seed"])[None]
    x = synth.make_source(dims, p["x_seed"])[None]
    print_case(test="golden_c4_vjp", prec=prec, recompute=recompute, dims=dims, k=k)
    lat = ovderiv.Lattice(dims, precision=ovderiv.FP64 if prec == "fp64" else ovderiv.MIXED,
                          basis_recompute=recompute)
    lat.set_links(dev(U))
    s, dm, F, _, _ = lat.sign_apply_vjp(dev(x), dev(b), mu, k, force=True, u1=True)
    assert lat.last_stats.basis_recomputed == int(recompute)
    drift = _coef_drift(lat, g, 0, k)
    th = host(lat.last_dsdtheta)
    F = host(F)
    lat.close()
    links = np.array(g["links"])
    Fmax = g["F_absmax"]
    e_s = _rel(s, complex(*g["s"]))
    e_dm = _rel(dm, complex(*g["ds_dmu"]))
    e_F = np.abs(F[links[:, 0], links[:, 1]] - _c(g["F_links"])).max() / Fmax
    e_th = np.abs(th[links[:, 0], links[:, 1]] - _c(g["u1_links"])).max() / Fmax
    print(f"  s {e_s:.2e}  ds/dmu {e_dm:.2e}  F {e_F:.2e}  i tr F {e_th:.2e}; coefficient drift {drift}",
          flush=True)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert max(e_s, e_dm, e_F, e_th) <= tol
    if prec == "fp64":
        assert drift[k] < 1e-8, drift
