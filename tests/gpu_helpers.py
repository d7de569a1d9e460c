"""Shared helpers of the GPU parity tests (inputs from synth, references from oracle)."""
import numpy as np
import torch

import synth
from oracle import dirac


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """Distance of a from the reference b: the larger of the relative 2-norm
    error and the largest element error relative to the largest element of b,
    so that a bound on it is a bound element by element as well."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    if a.shape != b.shape:
        raise ValueError(f"shape mismatch {a.shape} vs {b.shape}")
    norm = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    elem = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300) if b.size else 0.0
    return max(norm, elem)


def ops(U, dims, mu, dU=None):
    """Oracle operators on flat vectors: H, H^dag, dH, dH^dag (mu or link direction)."""
    h = lambda v: dirac.flat(dirac.apply_h(U, v, dims, mu))
    hd = lambda v: dirac.flat(dirac.apply_hdag(U, v, dims, mu))
    if dU is None:
        dh = lambda v: dirac.flat(dirac.apply_dh_dmu(U, v, dims, mu))
        dhd = lambda v: -dirac.flat(dirac.apply_dh_dmu(U, v, dims, -mu))
    else:
        dh = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, dims, mu))
        dhd = lambda v: dirac.flat(dirac.apply_dh_dlink(dU, v, dims, -mu))
    return h, hd, dh, dhd


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def noise_sensitivity(run, trials=3, rel_noise=1e-16, seed=0):
    """How far the oracle's own result moves when every operator application is
    perturbed by relative noise at the rounding level: run(wrap) must compute
    the result with each operator callable f replaced by wrap(f).  Returns the
    largest relative change over a few trials.  Near a Lanczos breakdown the
    recurrence amplifies rounding, and this sets how closely any two FP64
    implementations (different summation orders) can agree."""
    rng = np.random.default_rng(seed)
    ref = np.asarray(run(lambda f: f)).ravel()

    def wrap(f):
        def g(v):
            y = f(v)
            return y * (1.0 + rel_noise * rng.standard_normal(y.shape))
        return g

    out = 0.0
    for _ in range(trials):
        y = np.asarray(run(wrap)).ravel()
        out = max(out, np.linalg.norm(y - ref) / np.linalg.norm(ref))
    return out
