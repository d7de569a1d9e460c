"""Host-side small dense algebra of the eigensolver (csrc/dense.hpp), built
with g++ and checked against numpy: eigenvalues of random, triangular,
Hermitian and defective-looking matrices, eigenvector residuals and the
inverse.  No GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("dense") / "dense_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "host", "dense_check.cpp"), "-o", out],
                   check=True)
    return out


def _run(exe, A):
    n = A.shape[0]
    txt = f"{n}\n" + "\n".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in A.ravel()) + "\n"
    r = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True)
    lines = r.stdout.strip().split("\n")
    w = np.array([complex(*map(float, ln.split())) for ln in lines[:n]])
    vals = {ln.split()[0]: float(ln.split()[1]) for ln in lines[n:]}
    return w, vals


def _match(w, ref):
    """max distance between two eigenvalue multisets (greedy nearest match)"""
    ref = list(ref)
    d = 0.0
    for z in w:
        i = int(np.argmin([abs(z - r) for r in ref]))
        d = max(d, abs(z - ref.pop(i)))
    return d


@pytest.mark.parametrize("n,kind", [(1, "random"), (7, "random"), (60, "random"), (40, "hermitian"),
                                    (30, "triangular"), (24, "jordanlike"), (50, "lowrank")])
def test_dense_eig_against_numpy(exe, n, kind):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if kind == "hermitian":
        A = A + A.conj().T
    elif kind == "triangular":
        A = np.triu(A)
    elif kind == "jordanlike":      # eigenvalue 2 with a near-Jordan block, then the rest
        A = np.triu(A) * 1e-3
        A[np.arange(n), np.arange(n)] = np.r_[np.full(4, 2.0), rng.standard_normal(n - 4)]
        A[np.arange(3), np.arange(1, 4)] = 1.0
    elif kind == "lowrank":         # a zero eigenvalue of multiplicity n - 5
        B = rng.standard_normal((n, 5)) + 1j * rng.standard_normal((n, 5))
        A = B @ (rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n)))
    w, vals = _run(exe, A)
    ref = np.linalg.eigvals(A)
    scale = max(1.0, np.abs(A).max())
    tol = 1e-3 if kind == "jordanlike" else 1e-10 * scale * n   # a Jordan-like block splits as eps^(1/4)
    assert _match(w, ref) < tol
    if kind != "jordanlike" and kind != "lowrank":
        assert vals["residual"] < 1e-11 * scale * n
    if kind in ("random", "hermitian", "triangular"):
        assert 0 <= vals["inverse"] < 1e-8
