"""Benchmark of the hot path: d<x|sgn(H(mu))|b>/dmu by two-sided Lanczos on the
block matrix (eq. 6-7 of the paper), at 14 x 14^3, k = 400, mu = 0.3, on one
MI355X, plus the Dw.v stencil bandwidth.

One step = one call of ovd_sign_apply_deriv over a batch of `nrhs` synthetic
(x, b) pairs in the storage-free scalar mode: k fused Lanczos steps on the GPU,
sgn(T_k) e_1, and the scalar <x|d sgn(H) b> per pair.  Inputs are resident in
HBM before the timed region.  value = derivative evaluations per second.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "d⟨x|sgn(H(μ))|b⟩/dμ evals/s at 14^4,k=400; Dw·v HBM GB/s vs peak"


def step_bytes_per_site(prec_bytes: int, nrhs: int) -> float:
    """Algorithmic HBM bytes per lattice site per fused Lanczos step (block system).

    Per right-hand side: 3 inputs x 2 sides x 2 halves x 12 complex read (the
    Lanczos update a X + b Y + c Z), 2 outputs x 2 sides x 2 halves x 12 complex
    written, the projection vector x (12 complex) read; the 4 x 9 complex links
    once per site per launch.  Complex = 2 * prec_bytes.
    """
    c = 2 * prec_bytes
    per_rhs = (3 * 2 * 2 * 12 + 2 * 2 * 2 * 12 + 12) * c
    links = 4 * 9 * c
    return per_rhs + links / nrhs


def dwv_bytes_per_site(prec_bytes: int) -> float:
    """Dw.v: read 12 complex + 4 x 9 link complex, write 12 complex per site."""
    return (12 + 36 + 12) * 2 * prec_bytes


def run_gpu(args):
    import numpy as np
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    U = synth.make_links(dims, args.eps, 1611)
    prec = ovderiv.MIXED if args.precision == "mixed" else ovderiv.FP64
    lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec)
    lat.set_links(torch.from_numpy(U).cuda())
    n = args.nrhs
    b = torch.from_numpy(synth.make_sources(dims, n, 4000)).cuda()
    x = torch.from_numpy(synth.make_sources(dims, n, 5000)).cuda()
    mus = [args.mu] * n
    for _ in range(args.warmup):
        lat.sign_apply_deriv(b, mus, args.k, x=x, want_vectors=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_lanczos = 0.0
    ms_sign = 0.0
    vals = None
    for _ in range(args.steps):
        _, _, vals = lat.sign_apply_deriv(b, mus, args.k, x=x, want_vectors=False)
        ms_lanczos += lat.last_stats.ms_lanczos
        ms_sign += lat.last_stats.ms_small_sign
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals = n * args.steps / dt
    pb = 4 if prec == ovderiv.MIXED else 8
    per_launch_ms = ms_lanczos / (args.steps * args.k)
    bytes_launch = step_bytes_per_site(pb, n) * V * n
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    out = {
        "evals_per_s": evals,
        "ms_per_step": 1e3 * dt / args.steps,
        "ms_lanczos_per_step": ms_lanczos / args.steps,
        "ms_small_sign_per_step": ms_sign / args.steps,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "tsl_step_kernel",
            "bytes_per_launch": bytes_launch,
            "us_per_launch": round(per_launch_ms * 1e3, 2),
        },
        "xdy0": [vals[0].real, vals[0].imag],
        "min_margin": lat.last_stats.min_margin,
        "sign_check": lat.last_stats.sign_check,
    }
    # Dw.v bandwidth: nrhs fields per launch so that the traffic exceeds the 256 MB MALL
    nd = args.dwv_nrhs
    src = torch.from_numpy(synth.make_sources(dims, 1, 6000)).cuda().repeat(nd, 1, 1, 1).contiguous()
    dw = {}
    for pname, pv in (("fp64", ovderiv.FP64), ("fp32", ovderiv.MIXED)):
        l2 = ovderiv.Lattice(dims, m0=args.m0, precision=pv)
        l2.set_links(torch.from_numpy(U).cuda())
        l2.apply_op(ovderiv.OP_DW, args.mu, src)
        ms = []
        for _ in range(5):
            l2.apply_op(ovderiv.OP_DW, args.mu, src)
            ms.append(l2.last_ms)
        ms_med = sorted(ms)[len(ms) // 2]
        pbb = 8 if pv == ovderiv.FP64 else 4
        byt = nd * V * (24 * 2 * pbb) + 36 * 2 * pbb * V
        dw[pname] = {"gbs": round(byt / (ms_med * 1e-3) / 1e9, 1), "ms": round(ms_med, 4), "nrhs": nd,
                     "bytes": byt, "frac": round(byt / (ms_med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        l2.close()
    out["dw_v"] = dw
    lat.close()
    return out


def run_cpu_baseline(args, nsteps):
    """The oracle, as it stands, on a bounded sample: `nsteps` of the k block
    Lanczos steps at the full lattice size plus one k x k Schur sign, scaled
    to evaluations per second."""
    import numpy as np

    import synth
    from oracle import dirac, matfun, tsl

    dims = tuple(args.dims)
    mu = args.mu
    U = synth.make_links(dims, args.eps, 1611)
    b = synth.make_source(dims, 4000).ravel()
    x = synth.make_source(dims, 5000).ravel()
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, args.m0))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, args.m0))
    dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, dims, mu))
    dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, dims, -mu))
    n = b.size
    op, op_h = tsl.block_ops(h, hd, dh, dhd, n)
    psi = np.concatenate([np.zeros(n, complex), b])
    phi = tsl.block_left_start(psi, n)
    xx = np.concatenate([x, np.zeros(n, complex)])
    t0 = time.perf_counter()
    tsl.lanczos(op, op_h, psi, phi, nsteps, keep_basis=False, proj=xx)
    t_step = (time.perf_counter() - t0) / nsteps
    rng = np.random.default_rng(0)
    T = np.diag(rng.choice([-1, 1], args.k) * rng.uniform(0.5, 4, args.k) + 0.1j * rng.standard_normal(args.k))
    T = T + np.diag(0.3 * rng.standard_normal(args.k - 1), 1) + np.diag(0.3 * rng.standard_normal(args.k - 1), -1)
    t1 = time.perf_counter()
    matfun.sign_schur(T)
    t_sign = time.perf_counter() - t1
    t_eval = args.k * t_step + t_sign
    return {
        "value": 1.0 / t_eval,
        "unit": "evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nsteps} of {args.k} block Lanczos steps at {'x'.join(map(str, dims))} "
                  f"({t_step:.2f} s/step, single-threaded numpy) + one {args.k}x{args.k} Schur sign "
                  f"({t_sign:.2f} s), scaled to one evaluation",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--k", type=int, default=400)
    ap.add_argument("--mu", type=float, default=0.3)
    ap.add_argument("--eps", type=float, default=0.4)
    ap.add_argument("--m0", type=float, default=-1.5)
    ap.add_argument("--dims", type=int, nargs=4, default=[14, 14, 14, 14])
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--dwv-nrhs", type=int, default=48)
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this path has no multi-GPU form "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    g = run_gpu(args)
    cpu = None if args.no_cpu_baseline else run_cpu_baseline(args, args.cpu_steps)
    res = {
        "metric": METRIC,
        "value": round(g["evals_per_s"], 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"d<x|sgn(H(mu))|b>/dmu, two-sided Lanczos on the block matrix, "
                        f"{'x'.join(map(str, args.dims))} lattice, SU(3) links eps={args.eps}, m0={args.m0}, "
                        f"mu={args.mu}, k={args.k}, no deflation, storage-free scalar mode",
            "lattice": args.dims,
            "k": args.k,
            "mu": args.mu,
            "nrhs_per_step": args.nrhs,
            "precision": args.precision,
            "deflation": 0,
        },
        "roofline": g["roofline"],
        "cpu_baseline": cpu,
        "detail": {
            "ms_lanczos_per_step": round(g["ms_lanczos_per_step"], 3),
            "ms_small_sign_per_step": round(g["ms_small_sign_per_step"], 3),
            "dw_v": g["dw_v"],
            "min_margin": g["min_margin"],
            "sign_check": g["sign_check"],
            "xdy_first": g["xdy0"],
        },
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
