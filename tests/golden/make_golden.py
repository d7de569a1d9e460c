"""Writes the stored oracle references of the full-size GPU parity tests.

Every value in ``tests/golden/*.json`` comes from this script, which calls
only ``oracle/`` (the CPU FP64 reference) and ``synth/`` (the seeded input
generators); nothing here comes from, or calls, the GPU library.  The oracle
needs minutes to hours for hundreds of block-Lanczos steps at these lattice
sizes, far too long for a test, so the results are computed once here and
read by ``tests/test_gpu_golden.py``.

What is computed (the paper's hot path at the workload sizes):
  * (case c4_vjp) the gradient of s = <x|sgn(H(mu))|b> at the headline size:
    s, ds/dmu and the force F on every link from the bilinear two-sided
    Lanczos run (left start x, right start b) with the Frechet derivative of
    sgn(T_k) (the gradient form built on Sec. 2; not in the paper), stored at
    64 sampled links with i tr F (the U(1) derivative of Sec. 4-5), the
    largest |F| entry and the Lanczos coefficients;
  * Sec. 2, eq. 6-7: the derivative d/dt sgn(H(mu)) b, and sgn(H(mu)) b, as
    the Krylov-Ritz approximation of sgn(B) (0; b) for the block matrix
    B = [[H, dH], [0, H]], k two-sided Lanczos steps (the closing part of
    Sec. 2), with the left start (b; b);
  * the storage-free scalar <x | d sgn(H) b>;
  * Sec. 2 (closing part): the plain sgn(H(mu)) b with k steps (C4 only);
  * the Lanczos coefficients alpha, beta, delta of every step (the entries of
    T_k), so that the GPU run can be compared step by step.

Stored per case: the parameters, <x|dy>, <x|y>, the 2-norms of y and dy, both
vectors at 64 sites drawn with a fixed seed (all 12 components), and the
coefficients; for the short, unconverged 6^4 run of the uneven batch also the
oracle's own sensitivity of <x|dy> to relative noise of 1e-16 and 1e-7 in
every operator application (the precision its arithmetic can determine).

Usage:  python tests/golden/make_golden.py [case ...]   (default: all cases;
        one process per case, at most 6 at once)
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dirac, matfun, tsl, vjp  # noqa: E402

NSITES = 64
SITE_SEED = 99


def _case(dims, eps, link_seed, mu, k, b_seed, x_seed, direction="mu", dir_seed=None, vectors=True,
          plain=False, cite="Sec. 2, eq. 6-7 (block derivative) with the two-sided Lanczos of Sec. 2"):
    return dict(dims=list(dims), eps=eps, link_seed=link_seed, mu=mu, k=k, b_seed=b_seed, x_seed=x_seed,
                direction=direction, dir_seed=dir_seed, vectors=vectors, plain=plain, m0=-1.5, cite=cite)


def _c5_mus():
    """mu of the two sources of each lattice of the uneven-batch test: drawn in
    lattice order (6^4, 10^4, 16^4, 20 x 20^3) from one generator."""
    rng = np.random.default_rng(1616)
    return [list(rng.uniform(0.0, 0.5, 2)) for _ in range(4)]


def cases():
    c = {}
    # 14 x 14^3, eps = 0.4, mu = 0.3, k = 400: the headline workload, bench seeds
    # (links 1611, source i: b seed 4000 + i, x seed 5000 + i); sources 0 and 7
    for r in (0, 7):
        c[f"c4_r{r}"] = _case((14, 14, 14, 14), 0.4, 1611, 0.3, 400, 4000 + r, 5000 + r, plain=True)
    # 8^4, eps = 0.5, k = 200; mu in {0, 0.2, 0.4}; the mu direction and a random
    # su(3) link direction X = i sum_a eta_a lambda_a / 2 (dU = X U)
    for mu in (0.0, 0.2, 0.4):
        for d in ("mu", "link"):
            c[f"c2_mu{mu:.1f}_{d}"] = _case((8, 8, 8, 8), 0.5, 1613, mu, 200, 1614, 1617, direction=d,
                                            dir_seed=1615 if d == "link" else None)
    # 12^4, k = 300: sources 0 (mu = 0.1) and 63 (mu = 0.4) of the 64-source batch
    # (16 sources, b seed 1700 + i, x seed 1800 + i, repeated for each mu)
    c["c3_r0"] = _case((12, 12, 12, 12), 0.4, 1612, 0.1, 300, 1700, 1800, vectors=False)
    c["c3_r63"] = _case((12, 12, 12, 12), 0.4, 1612, 0.4, 300, 1715, 1815, vectors=False)
    # uneven batch: 10^4 (k = 250) both sources, 16^4 (k = 400) source 0; the 6^4 and
    # 20 x 20^3 lattices below
    mus = _c5_mus()
    for r in range(2):
        c[f"c5_10_r{r}"] = _case((10, 10, 10, 10), 0.4, 1621, float(mus[1][r]), 250, 1640 + r, 1690 + r,
                                 vectors=False)
    c["c5_16_r0"] = _case((16, 16, 16, 16), 0.4, 1622, float(mus[2][0]), 400, 1650, 1700, vectors=False)
    # and source 0 of the smallest (6^4, k = 150) and the largest (20 x 20^3, k = 500) lattice
    c["c5_6_r0"] = dict(_case((6, 6, 6, 6), 0.4, 1620, float(mus[0][0]), 150, 1630, 1680, vectors=False),
                        sensitivity=True)
    c["c5_20_r0"] = _case((20, 20, 20, 20), 0.4, 1623, float(mus[3][0]), 500, 1660, 1710, vectors=False)
    # the gradient at the headline size: source 0 of the bench (b seed 4000, x seed 5000)
    c["c4_vjp"] = dict(_case((14, 14, 14, 14), 0.4, 1611, 0.3, 400, 4000, 5000,
                             cite="gradient of <x|sgn(H)|b>: bilinear two-sided Lanczos (Sec. 2) and the "
                                  "Frechet derivative of sgn(T_k) (eq. 6 applied to T_k)"), kind="vjp")
    return c


def _ops(U, dims, mu, m0, dU=None):
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0))
    if dU is None:
        dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, dims, mu))
        dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, dims, -mu))
    else:
        dh = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, dims, mu))
        dhd = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, dims, -mu))
    return h, hd, dh, dhd


def _cl(a):
    """complex array -> nested [re, im] lists (17 significant digits survive JSON)"""
    a = np.asarray(a, dtype=np.complex128)
    return np.stack([a.real, a.imag], axis=-1).tolist()


def _coeffs(L, k):
    """T_k entries in the library's convention: alpha[0..k-1]; beta[j], delta[j]
    for j = 1..k-1 (super- and sub-diagonal); index 0 is not part of T_k."""
    beta = np.array(L["beta"][:k])
    delta = np.array(L["delta"][:k])
    beta[0] = 0.0
    delta[0] = 0.0
    return dict(alpha=_cl(L["alpha"][:k]), beta=_cl(beta), delta=_cl(delta))


def _sensitivity(h, hd, dh, dhd, b, x, k, rel_noise, trials=3, seed=0):
    """Largest relative change of <x|dy> over a few runs in which every operator
    application is multiplied element-wise by (1 + rel_noise g), g standard
    normal: how precisely the k-step result is determined by arithmetic of
    that relative accuracy (1e-16: FP64; 1e-7: FP32 vectors and stencil)."""
    n = b.size
    rng = np.random.default_rng(seed)

    def scalar(wrap):
        op, op_h = tsl.block_ops(wrap(h), wrap(hd), wrap(dh), wrap(dhd), n)
        psi = np.concatenate([np.zeros(n, dtype=np.complex128), b])
        xx = np.concatenate([x, np.zeros(n, dtype=np.complex128)])
        L = tsl.lanczos(op, op_h, psi, tsl.block_left_start(psi, n), k, keep_basis=False, proj=xx)
        return L["norm"] * np.dot(L["proj"], tsl.ritz_coeffs(L["T"]))

    def noisy(f):
        def g(v):
            y = f(v)
            return y * (1.0 + rel_noise * rng.standard_normal(y.shape))
        return g

    ref = scalar(lambda f: f)
    return max(abs(scalar(noisy) - ref) / abs(ref) for _ in range(trials))


def run_case(name: str, p: dict) -> dict:
    t0 = time.time()
    dims = tuple(p["dims"])
    mu, k, m0 = p["mu"], p["k"], p["m0"]
    V = synth.volume(dims)
    U = synth.make_links(dims, p["eps"], p["link_seed"])
    b = synth.make_source(dims, p["b_seed"]).ravel()
    x = synth.make_source(dims, p["x_seed"]).ravel()
    dU = None
    if p["direction"] == "link":
        dU = dirac.link_tangent(synth.make_su3_direction(dims, p["dir_seed"]), U)
    h, hd, dh, dhd = _ops(U, dims, mu, m0, dU)
    n = b.size
    op, op_h = tsl.block_ops(h, hd, dh, dhd, n)
    psi = np.concatenate([np.zeros(n, dtype=np.complex128), b])
    phi = tsl.block_left_start(psi, n)
    xx = np.concatenate([x, np.zeros(n, dtype=np.complex128)])
    out = dict(case=name, params=p, generator="tests/golden/make_golden.py (oracle/ and synth/ only)")
    sites = np.sort(np.random.default_rng(SITE_SEED).choice(V, NSITES, replace=False))
    if p["vectors"]:
        L = tsl.lanczos(op, op_h, psi, phi, k, proj=xx)
        c = tsl.ritz_coeffs(L["T"])
        yb = L["norm"] * (L["V"] @ c)
        del L["V"], L["W"]
        dy, y = yb[:n], yb[n:]
        out.update(sites=sites.tolist(), dy_sites=_cl(dy.reshape(V, 12)[sites]), y_sites=_cl(y.reshape(V, 12)[sites]),
                   dy_norm=float(np.linalg.norm(dy)), y_norm=float(np.linalg.norm(y)), xdy=_cl(np.vdot(x, dy)),
                   xy=_cl(np.vdot(x, y)))
        # the storage-free form of the same scalar: |psi| sum_j c_j <x|v_j>
        out["xdy_storage_free"] = _cl(L["norm"] * np.dot(L["proj"], c))
    else:
        L = tsl.lanczos(op, op_h, psi, phi, k, keep_basis=False, proj=xx)
        c = tsl.ritz_coeffs(L["T"])
        out["xdy"] = _cl(L["norm"] * np.dot(L["proj"], c))
    out.update(_coeffs(L, k))
    out["min_margin"] = float(L["min_margin"])
    if p.get("sensitivity"):
        out["sensitivity"] = {str(rn): float(_sensitivity(h, hd, dh, dhd, b, x, k, rn)) for rn in (1e-16, 1e-7)}
    if p["plain"]:
        Lp = tsl.lanczos(h, hd, b, b, k, proj=x)
        cp = tsl.ritz_coeffs(Lp["T"])
        yp = Lp["norm"] * (Lp["V"] @ cp)
        del Lp["V"], Lp["W"]
        out["plain"] = dict(cite="Sec. 2 (closing part): sgn(H) b by two-sided Lanczos, left start b",
                            y_sites=_cl(yp.reshape(V, 12)[sites]), y_norm=float(np.linalg.norm(yp)),
                            xy=_cl(np.vdot(x, yp)), **_coeffs(Lp, k))
    out["oracle_seconds"] = round(time.time() - t0, 1)
    return out


def run_vjp_case(name: str, p: dict) -> dict:
    t0 = time.time()
    dims = tuple(p["dims"])
    V = synth.volume(dims)
    U = synth.make_links(dims, p["eps"], p["link_seed"])
    b = synth.make_source(dims, p["b_seed"]).ravel()
    x = synth.make_source(dims, p["x_seed"]).ravel()
    s, ds_dmu, F, L = vjp.krylov_vjp(U, dims, p["mu"], x, b, p["k"], m0=p["m0"])
    rng = np.random.default_rng(SITE_SEED)
    links = np.stack([rng.integers(0, 4, NSITES), np.sort(rng.choice(V, NSITES, replace=False))], axis=1)
    Fs = F[links[:, 0], links[:, 1]]
    th = vjp.u1_derivative(F)[links[:, 0], links[:, 1]]
    out = dict(case=name, params=p, generator="tests/golden/make_golden.py (oracle/ and synth/ only)",
               s=_cl(s), ds_dmu=_cl(ds_dmu), links=links.tolist(), F_links=_cl(Fs), u1_links=_cl(th),
               F_absmax=float(np.abs(F).max()), F_norm=float(np.linalg.norm(F)), min_margin=float(L["min_margin"]))
    out.update(_coeffs(L, p["k"]))
    out["oracle_seconds"] = round(time.time() - t0, 1)
    return out


def _work(item):
    name, p = item
    res = run_vjp_case(name, p) if p.get("kind") == "vjp" else run_case(name, p)
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(res, f, separators=(",", ":"))
        f.write("\n")
    print(f"{name}: written in {res['oracle_seconds']} s", flush=True)
    return name


def main(argv):
    allc = cases()
    names = argv or list(allc)
    for nme in names:
        if nme not in allc:
            raise SystemExit(f"unknown case {nme}; known: {', '.join(allc)}")
    # the heavy cases first, so that they start at once
    names.sort(key=lambda n_: -np.prod(allc[n_]["dims"]) * allc[n_]["k"])
    with mp.get_context("fork").Pool(min(6, len(names))) as pool:
        for _ in pool.imap_unordered(_work, [(n_, allc[n_]) for n_ in names]):
            pass


if __name__ == "__main__":
    main(sys.argv[1:])
