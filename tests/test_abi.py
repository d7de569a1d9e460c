"""The C-ABI library builds, loads and exports every symbol include/ovderiv.h declares (no GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ovderiv.h")
LIB = os.path.join(ROOT, "paper_1611_00195_amd", "libovderiv.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ovd_[a-z_]+)\s*\(", txt)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_1611_00195_amd import build
        build.build(verbose=False)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ovd_create_lattice", "ovd_set_links", "ovd_set_deflation", "ovd_sign_apply",
              "ovd_sign_apply_deriv", "ovd_sign_apply_vjp"):
        assert n in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in _declared():
        assert re.search(rf"\bT {n}\b", out), n


def test_binding_lists_the_same_symbols():
    from paper_1611_00195_amd import ovderiv
    assert sorted(ovderiv.EXPORTS) == _declared()


def test_invalid_arguments_rejected_without_gpu_work():
    """Argument checks happen before any device call."""
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    lib.ovd_create_lattice.restype = ctypes.c_int
    h = ctypes.c_void_p()
    bad = (ctypes.c_int * 4)(4, 4, 1, 4)
    assert lib.ovd_create_lattice(bad, ctypes.c_double(-1.5), ctypes.c_double(1.0), -1, None, None,
                                  ctypes.byref(h)) == -1
    ok = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.ovd_create_lattice(ok, ctypes.c_double(-1.5), ctypes.c_double(0.5), -1, None, None,
                                  ctypes.byref(h)) == -1


def test_bad_options_and_small_sign_arguments_rejected():
    """Option ranges and the arguments of ovd_tridiag_sign are checked before
    any device call."""
    _ensure_built()
    from paper_1611_00195_amd import ovderiv
    lib = ctypes.CDLL(LIB)
    lib.ovd_create_lattice.restype = ctypes.c_int
    h = ctypes.c_void_p()
    ok = (ctypes.c_int * 4)(4, 4, 4, 4)
    base = dict(precision=0, left_start=0, breakdown_tol=1e-14, quad_step=0.1, step_timing=0, use_graph=1,
                autotune=1, shape_map=-1, shape_gpb=0, shape_seq=-1, shape_rp=0, basis_recompute=-1,
                quad_max_levels=0, sign_method=0, nested_inner=0, mem_budget=0, eig_shift_max=0, batch_separate=0)
    for bad in (dict(quad_max_levels=21), dict(sign_method=2), dict(nested_inner=-1), dict(mem_budget=-5),
                dict(precision=3), dict(eig_shift_max=-1), dict(batch_separate=2)):
        opt = ovderiv._Options(**{**base, **bad})
        assert lib.ovd_create_lattice(ok, ctypes.c_double(-1.5), ctypes.c_double(1.0), -1, ctypes.byref(opt), None,
                                      ctypes.byref(h)) == -1, bad
    lib.ovd_tridiag_sign.restype = ctypes.c_int
    a = (ctypes.c_double * 8)()
    assert lib.ovd_tridiag_sign(0, 4, a, a, a, None, a, None, None) == -1
    assert lib.ovd_tridiag_sign(1, 0, a, a, a, None, a, None, None) == -1
    assert lib.ovd_tridiag_sign(1, 4, None, a, a, None, a, None, None) == -1
