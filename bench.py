"""Benchmark of the hot path: d<x|sgn(H(mu))|b>/dmu by two-sided Lanczos on the
block matrix (eq. 6-7 of the paper), at 14 x 14^3, k = 400, mu = 0.3, on one
MI355X, plus the Dw.v stencil bandwidth.

One step = one call of ovd_sign_apply_deriv over a batch of `nrhs` synthetic
(x, b) pairs in the storage-free scalar mode: the deflation projections of
the m = 40 eigenpairs of smallest |lambda| (and the derivatives of the first
6), k fused Lanczos steps on the GPU, sgn(T_k) e_1, and the scalar
<x|d sgn(H) b> per pair.  The deflation set is computed on the GPU before the
timed region (its time is reported separately); inputs are resident in HBM.
value = derivative evaluations per second.

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


def progress(msg: str) -> None:
    """One line on stderr per finished stage (long runs stay visibly alive)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stencil_bytes_per_site(prec_bytes: int, nrhs: int) -> float:
    """Algorithmic HBM bytes per lattice site per stencil launch (block system).

    Per right-hand side: vhat and what (2 halves each, 12 complex per half)
    read, A vhat and A^dag what written, the projection vector x (12 complex)
    read; the 4 x 9 complex links once per site per launch.  Complex =
    2 * prec_bytes.
    """
    c = 2 * prec_bytes
    per_rhs = (2 * 2 * 12 + 2 * 2 * 12 + 12) * c
    return per_rhs + 4 * 9 * c / nrhs


def update_bytes_per_site(prec_bytes: int) -> float:
    """Three-term update, per site and right-hand side: 3 inputs read and 1
    output written on both sides, 2 halves of 12 complex each."""
    return 2 * (3 + 1) * 2 * 12 * 2 * prec_bytes


def measured_traffic(pb: int, nrhs: int, shapes: str = ""):
    """HBM bytes per stencil launch from the committed rocprofv3 counter
    summary, if it was taken on the current stencil source and this workload,
    for the launch shape (XCD order, groups per block, paired or sequential
    form) that the autotuner kept in this run; else None."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1611_00195_amd", "csrc", "kernels_stencil.hip")
    path = os.path.join(ROOT, "profiles", "tsl_stencil_14x14cubed_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    kv = {}
    for line in open(path):
        if ":" in line:
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    # the tuned entry "tsl:d:1:<nrhs>=map<m>,gpb<G>[,seq|,march];" of this run
    run = re.search(rf"tsl:{'d' if pb == 8 else 'f'}:1:{nrhs}=map(\d+),gpb(\d+)(,seq|,march)?;", shapes)
    if kv.get("kernels_stencil_sha256_16") != digest or run is None:
        return None
    key = (f"bytes_per_launch_{'fp64' if pb == 8 else 'fp32'}_nrhs{nrhs}_map{run.group(1)}_gpb{run.group(2)}"
           f"{'_' + run.group(3)[1:] if run.group(3) else ''}")
    return float(kv[key]) if key in kv else None


def tuned_entry(shapes: str, pb: int, nrhs: int) -> str:
    """The d/dmu stencil's entry "tsl:<d|f>:1:<nrhs>=...;" of the tuned shapes, or ""."""
    import re
    m = re.search(rf"tsl:{'d' if pb == 8 else 'f'}:1:{nrhs}=[^;]*;", shapes)
    return m.group(0) if m else ""


def dwv_bytes_per_site(prec_bytes: int) -> float:
    """Dw.v: read 12 complex + 4 x 9 link complex, write 12 complex per site."""
    return (12 + 36 + 12) * 2 * prec_bytes


def time_form(args, U, prec, n, steps, warmup, V, step_timing=False, lat=None):
    """Time `steps` batched derivative evaluations of n sources at one precision.

    step_timing=False: the production path (the k Lanczos steps replayed as one
    HIP graph).  step_timing=True: launched one by one with HIP events around
    every stencil and update kernel on the library's stream, for the roofline.
    lat: a lattice already set up (links, deflation set), kept open."""
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    own = lat is None
    if own:
        lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec, step_timing=step_timing)
        lat.set_links(U)
    b = torch.from_numpy(synth.make_sources(dims, n, 4000)).cuda()
    x = torch.from_numpy(synth.make_sources(dims, n, 5000)).cuda()
    mus = [args.mu] * n
    for _ in range(warmup):
        lat.sign_apply_deriv(b, mus, args.k, x=x, want_vectors=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = {"ms_lanczos": 0.0, "ms_small_sign": 0.0, "ms_stencil": 0.0, "ms_update": 0.0}
    vals = None
    for _ in range(steps):
        _, _, vals = lat.sign_apply_deriv(b, mus, args.k, x=x, want_vectors=False)
        st = lat.last_stats
        for key in acc:
            acc[key] += getattr(st, key)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {key: v / steps for key, v in acc.items()}
    res.update(shapes=lat.tuned_shapes())
    res.update(evals_per_s=n * steps / dt, ms_per_step=1e3 * dt / steps, vals=vals,
               min_margin=lat.last_stats.min_margin, sign_check=lat.last_stats.sign_check)
    if own:
        lat.close()
    return res


def mixed_accuracy(args, U, n, dset=None):
    """Per-result error of the mixed-precision derivative against FP64 on the
    benchmark's sources and links: sgn(H)b and d/dmu sgn(H)b as vectors
    (relative 2-norm) and <x|dy> (relative, and relative to |x| |dy|), with
    the deflation set dset = (lam, R, L, dR, dL) when given."""
    import numpy as np
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    b = torch.from_numpy(synth.make_sources(dims, n, 4000)).cuda()
    x = torch.from_numpy(synth.make_sources(dims, n, 5000)).cuda()
    res = {}
    for prec in (ovderiv.FP64, ovderiv.MIXED):
        lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec)
        lat.set_links(U)
        if dset is not None:
            lam, R, L, dR, dL = dset
            lat.set_deflation(args.mu, lam, R, L, 0 if dR is None else dR.shape[0], dR, dL)
        y, dy, s = lat.sign_apply_deriv(b, [args.mu] * n, args.k, x=x)
        lat.close()
        res[prec] = (y.reshape(n, -1), dy.reshape(n, -1), np.array(s))
    nrm = lambda a: torch.linalg.vector_norm(a, dim=-1).cpu().numpy()
    (y6, dy6, s6), (y3, dy3, s3) = res[ovderiv.FP64], res[ovderiv.MIXED]
    ey = nrm(y3 - y6) / nrm(y6)
    ed = nrm(dy3 - dy6) / nrm(dy6)
    es = np.abs(s3 - s6) / np.abs(s6)
    en = np.abs(s3 - s6) / (nrm(x.reshape(n, -1)) * nrm(dy6))
    return {"y_rel_max": float(ey.max()), "dy_rel_max": float(ed.max()),
            "dy_rel_median": float(np.median(ed)), "xdy_rel_max": float(es.max()),
            "xdy_err_over_x_dy_max": float(en.max()),
            "dy_rel_per_source": [float("%.2e" % v) for v in ed]}


def run_gpu(args):
    import numpy as np
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    Uh = synth.make_links(dims, args.eps, 1611)
    U = torch.from_numpy(Uh).cuda()
    prec = ovderiv.MIXED if args.precision == "mixed" else ovderiv.FP64
    n = args.nrhs
    # the headline workload: the m eigenpairs of smallest |lambda| deflated
    # (eq. 8), the first l of them with their derivatives for the derivative
    # (eq. 9-11); the set is computed on the GPU once, outside the timed region
    defl = None
    lat_d = None
    if args.deflation > 0:
        lat_d = ovderiv.Lattice(dims, m0=args.m0, precision=prec)
        lat_d.set_links(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            lam, est = lat_d.compute_deflation(args.mu, args.deflation, args.defl_l)
            torch.cuda.synchronize()
            defl = {"m": args.deflation, "l": args.defl_l, "setup_s": round(time.perf_counter() - t0, 1),
                    "lambda_min_max_abs": [float(abs(lam[0])), float(abs(lam[-1]))],
                    "max_res": max(est["max_res_right"], est["max_res_left"]), "max_biorth": est["max_biorth"],
                    "arnoldi_cycles": [est["outer_right"], est["outer_left"]], "shift_iters": est["shift_iters"],
                    "max_shift_res": est["max_shift_res"]}
            progress(f"deflation set m={args.deflation} l={args.defl_l} in {defl['setup_s']} s")
        except Exception as e:   # no converged set: the undeflated run is the headline, and says why
            defl = {"m": args.deflation, "l": args.defl_l, "error": str(e)}
            lat_d.close()
            lat_d = None
    und = time_form(args, U, prec, n, args.steps, args.warmup, V)
    progress(f"undeflated form: {und['evals_per_s']:.2f} evals/s")
    main = und
    if lat_d is not None:
        main = time_form(args, U, prec, n, args.steps, args.warmup, V, lat=lat_d)
        dset = lat_d.get_deflation(args.mu) if not args.skip_forms else None
        lat_d.close()
        progress(f"deflated form: {main['evals_per_s']:.2f} evals/s")
        defl["undeflated_evals_per_s"] = round(und["evals_per_s"], 3)
        defl["max_rel_diff_xdy_vs_undeflated"] = max(abs(a - b) / abs(b) for a, b in zip(main["vals"], und["vals"]))
    # roofline: the same workload launched kernel by kernel with events
    prof = time_form(args, U, prec, n, max(1, min(args.steps, 2)), 0, V, step_timing=True)
    pb = 4 if prec == ovderiv.MIXED else 8
    st_ms = prof["ms_stencil"] / args.k                   # average stencil launch
    up_ms = prof["ms_update"] / (args.k - 1)              # average update launch
    bytes_launch = stencil_bytes_per_site(pb, n) * V * n
    achieved = bytes_launch / (st_ms * 1e-3) / 1e9
    up_bytes = update_bytes_per_site(pb) * V * n
    out = {
        "evals_per_s": main["evals_per_s"],
        "ms_per_step": main["ms_per_step"],
        "ms_lanczos_per_step": main["ms_lanczos"],
        "ms_lanczos_per_step_kernel_by_kernel": prof["ms_lanczos"],
        "ms_small_sign_per_step": main["ms_small_sign"],
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(pb, n, prof["shapes"]),
            "kernel": "tsl_march_kernel" if ",march;" in tuned_entry(prof["shapes"], pb, n) else "tsl_stencil_kernel",
            "launch_shape": prof["shapes"],
            "bytes_per_launch": bytes_launch,
            "us_per_launch": round(st_ms * 1e3, 2),
        },
        "update_kernel": {"bytes_per_launch": up_bytes, "us_per_launch": round(up_ms * 1e3, 2),
                          "gbs": round(up_bytes / (up_ms * 1e-3) / 1e9, 1)},
        # the whole Lanczos path: the algorithmic bytes of k stencils and k - 1
        # updates per call, over the call's wall time (deflation and sgn(T_k) included)
        "path": {"bytes_per_eval": (args.k * bytes_launch + (args.k - 1) * up_bytes) / n,
                 "gbs": round((args.k * bytes_launch + (args.k - 1) * up_bytes) / n * main["evals_per_s"] / 1e9, 1),
                 "frac": round((args.k * bytes_launch + (args.k - 1) * up_bytes) / n * main["evals_per_s"] / 1e9
                               / HBM_PEAK_GBS, 4)},
        "xdy0": [main["vals"][0].real, main["vals"][0].imag],
        "deflation": defl,
        "deflated": lat_d is not None or (defl is not None and "error" not in defl),
        "min_margin": main["min_margin"],
        "sign_check": main["sign_check"],
    }
    # the other forms: single-source FP64 (the plain path), and the batched
    # form in the other precision, with its error against FP64 on the same inputs
    forms = {}
    if not args.skip_forms:
        other = ovderiv.FP64 if prec == ovderiv.MIXED else ovderiv.MIXED
        single = time_form(args, U, ovderiv.FP64, 1, max(1, args.steps // 2), 1, V)
        msingle = time_form(args, U, ovderiv.MIXED, 1, max(1, args.steps // 2), 1, V)
        oth = time_form(args, U, other, n, max(1, args.steps // 2), 1, V)
        ref = main["vals"] if prec == ovderiv.FP64 else oth["vals"]
        mix = oth["vals"] if prec == ovderiv.FP64 else main["vals"]
        err = max(abs(a - b) / abs(b) for a, b in zip(mix, ref))
        # the batched mixed form at 32 sources (4 sources per XCD), against the
        # plain single-source FP64 path
        m32 = time_form(args, U, ovderiv.MIXED, 32, 2, 1, V)
        mixed_n = oth["evals_per_s"] if other == ovderiv.MIXED else main["evals_per_s"]
        forms = {
            "fp64_single_evals_per_s": round(single["evals_per_s"], 3),
            "mixed_single_evals_per_s": round(msingle["evals_per_s"], 3),
            ("mixed" if other == ovderiv.MIXED else "fp64") + f"_batched{n}_evals_per_s": round(oth["evals_per_s"], 3),
            "mixed_batched32_evals_per_s": round(m32["evals_per_s"], 3),
            "mixed_batched_over_fp64_single": {str(n): round(mixed_n / single["evals_per_s"], 3),
                                               "32": round(m32["evals_per_s"] / single["evals_per_s"], 3)},
            "mixed_vs_fp64_max_rel_err_xdy": err,
            "launch_shapes": {"fp64_single": single["shapes"], "mixed_single": msingle["shapes"],
                              ("mixed" if other == ovderiv.MIXED else "fp64") + f"_batched{n}": oth["shapes"],
                              "mixed_batched32": m32["shapes"]},
        }
    out["forms"] = forms
    if not args.skip_forms:
        # vector-level accuracy of the mixed form, undeflated and with the set
        acc = {"undeflated": mixed_accuracy(args, U, n)}
        if lat_d is not None:
            acc["deflated"] = mixed_accuracy(args, U, n, dset)
            del dset
        out["mixed_accuracy"] = acc
        progress("mixed accuracy done")
    if not args.skip_forms:
        out["vjp"] = time_vjp(args, U, V)
        vm = time_vjp(args, U, V, prec=ovderiv.MIXED)
        F64, F32 = out["vjp"].pop("F"), vm.pop("F")
        import torch as _t
        vm["max_rel_dev_from_fp64"] = {
            "s": abs(complex(*vm["s"]) - complex(*out["vjp"]["s"])) / abs(complex(*out["vjp"]["s"])),
            "ds_dmu": abs(complex(*vm["ds_dmu"]) - complex(*out["vjp"]["ds_dmu"])) / abs(complex(*out["vjp"]["ds_dmu"])),
            "force": float(_t.linalg.vector_norm(F32 - F64) / _t.linalg.vector_norm(F64)),
        }
        out["vjp_mixed"] = vm
        vr = time_vjp(args, U, V, recompute=True)
        Fr = vr.pop("F")
        vr["max_rel_dev_from_stored"] = {
            "s": abs(complex(*vr["s"]) - complex(*out["vjp"]["s"])) / abs(complex(*out["vjp"]["s"])),
            "force": float(_t.linalg.vector_norm(Fr - F64) / _t.linalg.vector_norm(F64)),
        }
        out["vjp_recompute"] = vr
        progress("gradient forms done")
        out["uneven"] = time_uneven(args)
        progress("uneven batch done")
    # achievable streaming bandwidth on this machine, for context beside the 8 TB/s
    # spec: a 1 GiB device-to-device copy (1 GiB read + 1 GiB written)
    src_c = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst_c = torch.empty_like(src_c)
    dst_c.copy_(src_c)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst_c.copy_(src_c)
    ev1.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = round(5 * 2 * (1 << 30) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
    del src_c, dst_c
    # Dw.v bandwidth: nrhs fields per launch so that the traffic exceeds the 256 MB MALL
    nd = args.dwv_nrhs
    src = torch.from_numpy(synth.make_sources(dims, 1, 6000)).cuda().repeat(nd, 1, 1, 1).contiguous()
    dw = {}
    for pname, pv in (("fp64", ovderiv.FP64), ("fp32", ovderiv.MIXED)):
        l2 = ovderiv.Lattice(dims, m0=args.m0, precision=pv)
        l2.set_links(U)
        l2.apply_op(ovderiv.OP_DW, args.mu, src)
        ms = []
        for _ in range(5):
            l2.apply_op(ovderiv.OP_DW, args.mu, src)
            ms.append(l2.last_ms)
        ms_med = sorted(ms)[len(ms) // 2]
        pbb = 8 if pv == ovderiv.FP64 else 4
        byt = nd * V * dwv_bytes_per_site(pbb) - (nd - 1) * V * 36 * 2 * pbb
        dw[pname] = {"gbs": round(byt / (ms_med * 1e-3) / 1e9, 1), "ms": round(ms_med, 4), "nrhs": nd,
                     "bytes": byt, "frac": round(byt / (ms_med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "cache": "cold: the launch's fields and links exceed the 256 MB last-level cache"}
        # warm: one field, repeated, whose field, result and links (37 MB in FP64) stay in that cache
        one = src[:1].contiguous()
        l2.apply_op(ovderiv.OP_DW, args.mu, one)
        ms1 = []
        for _ in range(21):
            l2.apply_op(ovderiv.OP_DW, args.mu, one)
            ms1.append(l2.last_ms)
        m1 = sorted(ms1)[len(ms1) // 2]
        b1 = V * dwv_bytes_per_site(pbb)
        dw[pname]["warm_1rhs"] = {"gbs": round(b1 / (m1 * 1e-3) / 1e9, 1), "ms": round(m1, 4), "bytes": b1,
                                  "frac": round(b1 / (m1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        l2.close()
    out["dw_v"] = dw
    return out


def time_vjp(args, U, V, prec=0, recompute=False):
    """The gradient of s = <x|sgn(H)|b> w.r.t. mu and all 4 V links (one source
    pair; both Krylov bases stored, or with recompute the right basis
    regenerated by a second Lanczos run): calls per second and the MFMA work
    of the Z = W M'^dag product (8 N k^2 flops)."""
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec, basis_recompute=recompute)
    lat.set_links(U)
    b = torch.from_numpy(synth.make_sources(dims, 1, 4000)).cuda()
    x = torch.from_numpy(synth.make_sources(dims, 1, 5000)).cuda()
    lat.sign_apply_vjp(x, b, args.mu, args.k, force=True, wirtinger=True)
    assert lat.last_stats.basis_recomputed == int(recompute)
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):   # median of 5 calls (single calls of tens of ms are noisy)
        t0 = time.perf_counter()
        s, dsdmu, F, _, _ = lat.sign_apply_vjp(x, b, args.mu, args.k, force=True, wirtinger=True)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    dt = sorted(ts)[len(ts) // 2]
    lat.close()
    return {"calls_per_s": round(1.0 / dt, 3), "ms_per_call": round(1e3 * dt, 2), "s": [s.real, s.imag],
            "ds_dmu": [dsdmu.real, dsdmu.imag], "precision": "fp64" if prec == 0 else "mixed", "k": args.k,
            "basis": "recomputed" if recompute else "stored", "zgemm_flops": 8.0 * 12 * V * args.k ** 2, "F": F}


def time_uneven(args):
    """Uneven batch: 12 derivative solves on each of 6^4, 10^4, 16^4 and 20x20^3
    (mu ~ U[0, 0.5], k = 150, 250, 400, 500 by size), one handle and stream per
    lattice, all four submitted together (ovd_sign_apply_deriv_batch), in the
    mixed precision and in FP64: with the Lanczos steps shared (one update and
    one stencil launch per step for every lattice still running) and, for
    comparison, with each lattice's steps on its own stream; per-solve
    deviation of mixed from FP64."""
    import numpy as np
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    shapes = [((6, 6, 6, 6), 150), ((10, 10, 10, 10), 250), ((16, 16, 16, 16), 400), ((20, 20, 20, 20), 500)]
    rng = np.random.default_rng(5000)
    inputs = []
    for i, (dims, k) in enumerate(shapes):
        U = torch.from_numpy(synth.make_links(dims, args.eps, 1611 + i)).cuda()
        b = torch.from_numpy(synth.make_sources(dims, 12, 6100 + 100 * i)).cuda()
        x = torch.from_numpy(synth.make_sources(dims, 12, 6150 + 100 * i)).cuda()
        mus = list(rng.uniform(0.0, 0.5, 12))
        inputs.append((dims, k, U, b, x, mus))

    def batch(prec, separate):
        jobs = []
        for dims, k, U, b, x, mus in inputs:
            lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec, stream=torch.cuda.Stream(),
                                  batch_separate=separate)
            lat.set_links(U)
            jobs.append((lat, b, mus, k, x))
        return jobs

    out = {}
    for name, prec in (("fp64", ovderiv.FP64), ("mixed", ovderiv.MIXED)):
        for separate in (False, True):
            jobs = batch(prec, separate)
            ovderiv.sign_apply_deriv_batch(jobs)          # warm-up: graphs and launch shapes
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ovderiv.sign_apply_deriv_batch(jobs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out[name + ("_separate" if separate else "")] = {"evals_per_s": round(48 / dt, 3), "s": round(dt, 3),
                                                             "vals": res}
            for j in jobs:
                j[0].close()
    errs = [[abs(a - b) / abs(b) for a, b in zip(ra, rb)] for ra, rb in zip(out["mixed"]["vals"], out["fp64"]["vals"])]
    dsep = max(abs(a - b) / abs(b) for ra, rb in zip(out["fp64"]["vals"], out["fp64_separate"]["vals"])
               for a, b in zip(ra, rb))
    return {"lattices": ["x".join(map(str, d)) for d, _ in shapes], "k": [k for _, k in shapes], "solves": 48,
            "mixed_evals_per_s": out["mixed"]["evals_per_s"], "fp64_evals_per_s": out["fp64"]["evals_per_s"],
            "form": "shared Lanczos steps: one update and one stencil launch per step for all lattices",
            "separate_streams": {"mixed_evals_per_s": out["mixed_separate"]["evals_per_s"],
                                 "fp64_evals_per_s": out["fp64_separate"]["evals_per_s"],
                                 "fp64_max_rel_diff_vs_shared": dsep},
            "mixed_vs_fp64_rel_err_max_per_lattice": [float(max(e)) for e in errs],
            "mixed_vs_fp64_rel_err_median_per_lattice": [float(np.median(e)) for e in errs],
            "note": "k = 150 on 6^4 and 250 on 10^4 leave the FP64 result itself unconverged at the 4e-3 level "
                    "for mu near 0.5; the mixed deviation there follows that truncation"}


def error_vs_k(args):
    """The analog of the paper's Fig. 1 on synthetic links: the Sec. 4 error
    estimates eps_A (the function) and eps_B (its mu-derivative) against the
    outer Krylov size k, without and with deflation (the 40 eigenpairs of
    smallest |lambda|; the derivative deflated with the paper's 6 pairs at
    14 x 14^3 and 2 at 6 x 18^3), for smooth (eps = 0.4) and rough (eps = 1.0)
    links.  The quadrature signs the Ritz matrices (the paper used its nested
    two-sided Lanczos; the nested option gives the same numbers within its
    inner accuracy).  Prints one JSON line."""
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    torch.cuda.set_device(0)
    ks = [50, 100, 150, 200, 250, 300, 350, 400]
    cases = [((14, 14, 14, 14), 0.300, 6), ((18, 18, 18, 6), 0.230, 2)]
    out = []
    for dims, mu, l in cases:
        for eps in args.eps_list:
            U = torch.from_numpy(synth.make_links(dims, eps, 1611)).cuda()
            phi = torch.from_numpy(synth.make_sources(dims, 1, 7000)).cuda()
            lat = ovderiv.Lattice(dims, m0=args.m0, eig_shift_max=args.eig_shift_max)
            lat.set_links(U)
            rec = {"lattice": "x".join(map(str, dims)), "mu": mu, "eps_links": eps, "m": 40, "l": l, "k": ks}
            rec["eps_A"] = [lat.sign_error_estimate(phi, mu, k)[0] for k in ks]
            rec["eps_B"] = [lat.deriv_error_estimate(phi, mu, k)[0] for k in ks]
            progress(f"error vs k {rec['lattice']} eps={eps}: undeflated done")
            t0 = time.perf_counter()
            try:
                lam, st = lat.compute_deflation(mu, 40, l)
                rec["setup_s"] = round(time.perf_counter() - t0, 1)
                rec["lambda_abs_min_max"] = [float(abs(lam[0])), float(abs(lam[-1]))]
                rec["eps_A_deflated"] = [lat.sign_error_estimate(phi, mu, k)[0] for k in ks]
                rec["eps_B_deflated"] = [lat.deriv_error_estimate(phi, mu, k)[0] for k in ks]
            except Exception as e:   # no converged set: recorded, the undeflated curve stands
                rec["deflation_error"] = str(e)
            progress(f"error vs k {rec['lattice']} eps={eps}: deflated done")
            lat.close()
            out.append(rec)
    print(json.dumps({"error_vs_k": out}))


# the stencil launch shapes the autotuner chooses among at 14^4 with 8 sources
# (groups per block, form: 0 paired, 1 sequential; with form 3, the
# time-marching form, the number of time segments); each in both XCD orders
COUNTER_SHAPES = ((8, 0), (1, 0), (2, 0), (1, 1), (2, 1), (1, 3), (2, 3), (4, 3))


def counters_run(args):
    """The workload of the committed counter summaries: the bench lattice and
    sources, 8 right-hand sides, 20 Lanczos steps, FP64 then mixed, in every
    launch shape the autotuner chooses among (each kernel in XCD order 0 and
    then order 1), then a 1 GiB device copy that calibrates the counters.
    The shapes are forced, since a profiler that serialises every dispatch
    distorts the tuner's timings; the bench then takes the counts of the
    shape its own run kept."""
    import torch

    import synth
    from paper_1611_00195_amd import ovderiv

    dims = tuple(args.dims)
    U = torch.from_numpy(synth.make_links(dims, args.eps, 1611)).cuda()
    b = torch.from_numpy(synth.make_sources(dims, 8, 4000)).cuda()
    x = torch.from_numpy(synth.make_sources(dims, 8, 5000)).cuda()
    for prec in (ovderiv.FP64, ovderiv.MIXED):
        for gpb, seq in COUNTER_SHAPES:
            for order in (0, 1):
                lat = ovderiv.Lattice(dims, m0=args.m0, precision=prec, shape=(order, gpb, seq))
                lat.set_links(U)
                lat.sign_apply_deriv(b, [args.mu] * 8, 20, x=x, want_vectors=False)
                torch.cuda.synchronize()
                lat.close()
    # calibration: a plain 1 GiB device-to-device copy (1 GiB read, 1 GiB written)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("counters run done", flush=True)


def _cpu_source_worker(job):
    """One source of the batch on one host core: the deflation projections of
    the block source (eq. 11, with stand-in eigen-data of the set's shape: the
    timing does not depend on the values) and `nsteps` block Lanczos steps of
    the oracle; returns (seconds of projections, seconds per step)."""
    dims, eps, mu, m0, nsteps, r, l = job
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import deflation, dirac, tsl

    with threadpool_limits(limits=1):
        U = synth.make_links(dims, eps, 1611)
        b = synth.make_source(dims, 4000 + r).ravel()
        x = synth.make_source(dims, 5000 + r).ravel()
        h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu, m0))
        hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu, m0))
        dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, dims, mu))
        dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, dims, -mu))
        n = b.size
        op, op_h = tsl.block_ops(h, hd, dh, dhd, n)
        psi = np.concatenate([np.zeros(n, complex), b])
        xx = np.concatenate([x, np.zeros(n, complex)])
        t_defl = 0.0
        if l > 0:
            rng = np.random.default_rng(r)
            R, L, dR, dL = (rng.standard_normal((n, l)) + 1j * rng.standard_normal((n, l)) for _ in range(4))
            t0 = time.perf_counter()
            proj, c_t, c_b = deflation.block_projector_apply(psi, R, L, dR, dL)
            psi = psi - proj
            exact = R @ c_t + dR @ c_b
            _ = np.vdot(x, exact)
            t_defl = time.perf_counter() - t0
        phi = tsl.block_left_start(psi, n)
        t0 = time.perf_counter()
        tsl.lanczos(op, op_h, psi, phi, nsteps, keep_basis=False, proj=xx)
        t_step = (time.perf_counter() - t0) / nsteps
    return t_defl, t_step


def run_cpu_baseline(args, nsteps):
    """The oracle, as it stands, on a bounded sample of the benchmark's
    workload on all the host cores: one process per core (at most the box's
    CPU share of 16), each with BLAS held to one thread and its own source
    (the batch's sources first); each does the deflation projections of its
    source and `nsteps` of the k block Lanczos steps at the full lattice
    size.  One k x k Schur sign is timed once.  Scaled to evaluations per
    second of all the processes together."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import matfun

    dims = tuple(args.dims)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = max(1, min(ncpu, 16))
    l = args.defl_l if args.deflation > 0 else 0
    jobs = [(dims, args.eps, args.mu, args.m0, nsteps, r, l) for r in range(procs)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_cpu_source_worker, jobs)
    wall = time.perf_counter() - t0
    t_defl = max(a for a, _ in res)
    t_step = max(b for _, b in res)
    rng = np.random.default_rng(0)
    T = np.diag(rng.choice([-1, 1], args.k) * rng.uniform(0.5, 4, args.k) + 0.1j * rng.standard_normal(args.k))
    T = T + np.diag(0.3 * rng.standard_normal(args.k - 1), 1) + np.diag(0.3 * rng.standard_normal(args.k - 1), -1)
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        matfun.sign_schur(T)
        t_sign = time.perf_counter() - t1
    t_eval = t_defl + args.k * t_step + t_sign          # one evaluation on one core
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": procs / t_eval,
        "unit": "evals/s",
        "cores": procs,
        "kind": "oracle",
        "cpu": model,
        "sample": f"{procs} sources side by side (the {args.nrhs} of the batch first), one process and one BLAS "
                  f"thread each, on {model} ({ncpu} cores available): per source the projections of the {l}-pair "
                  f"generalised deflation ({t_defl:.2f} s) and {nsteps} of {args.k} block Lanczos steps at "
                  f"{'x'.join(map(str, dims))} ({t_step:.2f} s/step, slowest process), plus one {args.k}x{args.k} "
                  f"Schur sign ({t_sign:.2f} s); scaled to one evaluation per process ({wall:.0f} s wall)",
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
    ap.add_argument("--deflation", type=int, default=40,
                    help="eigenpairs of smallest |lambda| deflated (0: none); computed on the GPU before timing")
    ap.add_argument("--defl-l", type=int, default=6,
                    help="of those, the pairs whose derivatives enter the deflated derivative")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-forms", action="store_true")
    ap.add_argument("--error-vs-k", action="store_true",
                    help="the Fig. 1 analog: Sec. 4 error estimates against k with and without deflation; "
                         "prints one JSON line and no benchmark line")
    ap.add_argument("--eig-shift-max", type=int, default=0,
                    help="iteration limit of the eigensolver's shifted solves in --error-vs-k (0: library default)")
    ap.add_argument("--eps-list", type=float, nargs="+", default=[0.4, 1.0],
                    help="link roughness values of --error-vs-k")
    ap.add_argument("--counters-run", action="store_true",
                    help="short fixed workload for rocprofv3 --pmc runs (8 sources, 20 Lanczos steps, "
                         "FP64 then mixed); prints one line and no JSON")
    ap.add_argument("--uneven-only", action="store_true",
                    help="only the uneven batch (48 solves on 6^4 .. 20x20^3, shared and separate forms); "
                         "prints its JSON record")
    ap.add_argument("--vjp-only", action="store_true",
                    help="only the gradient of <x|sgn(H)|b> (FP64 and mixed, bases stored); prints its JSON record")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this path has no multi-GPU form "
              "(independent solves would shard one group per GPU); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.counters_run:
        counters_run(args)
        return
    if args.error_vs_k:
        error_vs_k(args)
        return
    if args.uneven_only:
        import torch
        torch.cuda.set_device(0)
        rec = time_uneven(args)
        rec.pop("vals", None)
        print(json.dumps(rec), flush=True)
        return
    if args.vjp_only:
        import synth
        import torch
        torch.cuda.set_device(0)
        dims = tuple(args.dims)
        V = dims[0] * dims[1] * dims[2] * dims[3]
        U = torch.from_numpy(synth.make_links(dims, args.eps, 1611)).cuda()
        rec = {}
        for name, prec in (("fp64", 0), ("mixed", 1)):
            r = time_vjp(args, U, V, prec=prec)
            r.pop("F", None)
            rec[name] = r
        print(json.dumps(rec), flush=True)
        return
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
                        f"mu={args.mu}, k={args.k}, "
                        + (f"m={args.deflation} eigenpairs deflated (generalised deflation of the first "
                           f"{args.defl_l} for the derivative)" if g["deflated"] else "no deflation")
                        + ", storage-free scalar mode",
            "lattice": args.dims,
            "k": args.k,
            "mu": args.mu,
            "nrhs_per_step": args.nrhs,
            "precision": args.precision,
            "deflation": args.deflation if g["deflated"] else 0,
            "derivative_deflation_pairs": args.defl_l if g["deflated"] else 0,
        },
        "roofline": g["roofline"],
        "cpu_baseline": cpu,
        "detail": {
            "deflation": g["deflation"],
            "ms_lanczos_per_step": round(g["ms_lanczos_per_step"], 3),
            "ms_small_sign_per_step": round(g["ms_small_sign_per_step"], 3),
            "update_kernel": g["update_kernel"],
            "path": g["path"],
            "copy_1gib_gbs": g.get("copy_gbs"),
            "forms": g["forms"],
            "mixed_vs_fp64": g.get("mixed_accuracy"),
            "dw_v": g["dw_v"],
            "vjp": g.get("vjp"),
            "vjp_mixed": g.get("vjp_mixed"),
            "vjp_recompute": g.get("vjp_recompute"),
            "uneven_batch": g.get("uneven"),
            "min_margin": g["min_margin"],
            "sign_check": g["sign_check"],
            "xdy_first": g["xdy0"],
        },
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
