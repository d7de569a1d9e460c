"""Python binding of libovderiv (ctypes; argument marshalling only).

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, passes device pointers and the current torch stream, and
turns status codes into exceptions.  PyTorch provides device memory and
streams only.  If the library has not been built the import fails loudly:
there is no CPU fallback.

Names follow the C ABI (include/ovderiv.h): ``create_lattice``, ``set_links``,
``set_deflation``, ``sign_apply``, ``sign_apply_deriv``, ``sign_apply_vjp``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OVDERIV_LIB", os.path.join(_HERE, "libovderiv.so"))

OVD_OK, OVD_EINVAL, OVD_ENOMEM, OVD_EHIP, OVD_EBREAKDOWN, OVD_ENODEFL, OVD_ENAN, OVD_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
LEFT_SUM, LEFT_SAME = 0, 1
DIR_MU, DIR_LINK = 0, 1
OP_H, OP_DW, OP_DH_DMU, OP_DH_DLINK = 0, 1, 2, 3
SIGN_QUAD, SIGN_NESTED = 0, 1

EXPORTS = [
    "ovd_create_lattice", "ovd_destroy", "ovd_last_error", "ovd_set_stream", "ovd_set_links",
    "ovd_apply_op", "ovd_set_deflation", "ovd_clear_deflation", "ovd_sign_apply",
    "ovd_sign_apply_deriv", "ovd_sign_apply_vjp", "ovd_get_tridiag", "ovd_compute_deflation",
    "ovd_get_deflation", "ovd_sign_apply_deriv_batch", "ovd_get_tuned", "ovd_overlap_apply",
    "ovd_sign_error_estimate", "ovd_tridiag_sign", "ovd_block_sign_apply", "ovd_deriv_error_estimate",
    "ovd_sign_apply_deriv_noalloc",
]


class OvdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libovderiv status {status}: {msg}")
        self.status = status


class Breakdown(OvdError):
    pass


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("left_start", ctypes.c_int),
                ("breakdown_tol", ctypes.c_double), ("quad_step", ctypes.c_double),
                ("step_timing", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("shape_map", ctypes.c_int), ("shape_gpb", ctypes.c_int), ("shape_seq", ctypes.c_int),
                ("shape_rp", ctypes.c_int), ("basis_recompute", ctypes.c_int),
                ("quad_max_levels", ctypes.c_int), ("sign_method", ctypes.c_int), ("nested_inner", ctypes.c_int),
                ("mem_budget", ctypes.c_longlong), ("eig_shift_max", ctypes.c_int),
                ("batch_separate", ctypes.c_int)]


class _EigStats(ctypes.Structure):
    _fields_ = [("outer_right", ctypes.c_int), ("outer_left", ctypes.c_int),
                ("max_res_right", ctypes.c_double), ("max_res_left", ctypes.c_double),
                ("max_biorth", ctypes.c_double), ("shift_iters", ctypes.c_int),
                ("max_shift_res", ctypes.c_double), ("ms", ctypes.c_double)]


class _Dir(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dU", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("breakdown_step", ctypes.c_int), ("min_margin", ctypes.c_double),
                ("sign_check", ctypes.c_double), ("ms_lanczos", ctypes.c_double),
                ("ms_small_sign", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_stencil", ctypes.c_double), ("ms_update", ctypes.c_double), ("basis_recomputed", ctypes.c_int)]


class _Job(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("mu", ctypes.POINTER(ctypes.c_double)),
                ("dir", ctypes.c_void_p), ("k", ctypes.c_int), ("b", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("dy", ctypes.c_void_p), ("x", ctypes.c_void_p), ("xdy", ctypes.POINTER(ctypes.c_double)),
                ("st", ctypes.POINTER(_Stats)), ("status", ctypes.c_int)]


@dataclass
class Stats:
    k: int
    breakdown_step: int
    min_margin: float
    sign_check: float
    ms_lanczos: float
    ms_small_sign: float
    ms_total: float
    ms_stencil: float
    ms_update: float
    basis_recomputed: int = 0


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libovderiv is not built ({path} missing); run python -m paper_1611_00195_amd.build")
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ovd_create_lattice": (i, [ctypes.POINTER(ctypes.c_int), d, d, i, ctypes.POINTER(_Options), vp, ctypes.POINTER(vp)]),
        "ovd_destroy": (i, [vp]),
        "ovd_last_error": (ctypes.c_char_p, [vp]),
        "ovd_set_stream": (i, [vp, vp]),
        "ovd_set_links": (i, [vp, vp]),
        "ovd_apply_op": (i, [vp, i, d, ctypes.POINTER(_Dir), i, vp, vp, dp]),
        "ovd_set_deflation": (i, [vp, d, i, dp, vp, vp, i, vp, vp, ctypes.POINTER(_Dir)]),
        "ovd_clear_deflation": (i, [vp]),
        "ovd_overlap_apply": (i, [vp, i, dp, ctypes.POINTER(_Dir), i, vp, vp, vp, ctypes.POINTER(_Stats)]),
        "ovd_sign_error_estimate": (i, [vp, i, dp, i, vp, dp, ctypes.POINTER(_Stats)]),
        "ovd_get_tuned": (i, [vp, ctypes.c_char_p, i]),
        "ovd_sign_apply_deriv_batch": (i, [i, ctypes.POINTER(_Job)]),
        "ovd_get_deflation": (i, [vp, d, ctypes.POINTER(i), ctypes.POINTER(i), dp, vp, vp, vp, vp]),
        "ovd_compute_deflation": (i, [vp, d, i, i, ctypes.POINTER(_Dir), d, dp, ctypes.POINTER(_EigStats)]),
        "ovd_sign_apply": (i, [vp, i, dp, i, vp, vp, ctypes.POINTER(_Stats)]),
        "ovd_sign_apply_deriv": (i, [vp, i, dp, ctypes.POINTER(_Dir), i, vp, vp, vp, vp, dp, ctypes.POINTER(_Stats)]),
        "ovd_sign_apply_vjp": (i, [vp, d, i, vp, vp, dp, dp, vp, vp, vp, vp, ctypes.POINTER(_Stats)]),
        "ovd_get_tridiag": (i, [vp, i, i, dp, dp, dp]),
        "ovd_tridiag_sign": (i, [i, i, dp, dp, dp, ctypes.POINTER(_Options), dp, dp, vp]),
        "ovd_block_sign_apply": (i, [vp, i, dp, ctypes.POINTER(_Dir), i, vp, vp, vp, vp, ctypes.POINTER(_Stats)]),
        "ovd_deriv_error_estimate": (i, [vp, i, dp, ctypes.POINTER(_Dir), i, vp, dp, ctypes.POINTER(_Stats)]),
        "ovd_sign_apply_deriv_noalloc": (i, [vp, i, dp, ctypes.POINTER(_Dir), i, vp, vp, dp, ctypes.POINTER(_Stats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_field(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _dbl(arr):
    a = (ctypes.c_double * len(arr))(*arr)
    return a


class Lattice:
    """One lattice handle (``ovd_create_lattice``); links, deflation data and
    workspaces live on the current device."""

    def __init__(self, dims, m0=-1.5, r=1.0, t_bc=-1, precision=FP64, left_start=LEFT_SUM,
                 breakdown_tol=1e-14, quad_step=0.1, stream=None, step_timing=False, use_graph=True,
                 autotune=True, shape=None, basis_recompute=None, quad_max_levels=0, sign_method=SIGN_QUAD,
                 nested_inner=0, mem_budget=0, eig_shift_max=0, batch_separate=False):
        self.dims = tuple(int(d) for d in dims)
        self.V = 1
        for d in self.dims:
            self.V *= d
        self.precision = precision
        self._lib = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        opt = _Options(precision, left_start, breakdown_tol, quad_step, int(bool(step_timing)), int(bool(use_graph)),
                       int(bool(autotune)), -1 if shape is None else int(shape[0]),
                       0 if shape is None else int(shape[1]),
                       -1 if shape is None or len(shape) < 3 else int(shape[2]),
                       0 if shape is None or len(shape) < 4 else int(shape[3]),
                       -1 if basis_recompute is None else int(bool(basis_recompute)),
                       int(quad_max_levels), int(sign_method), int(nested_inner), int(mem_budget),
                       int(eig_shift_max), int(bool(batch_separate)))
        h = ctypes.c_void_p()
        dims_c = (ctypes.c_int * 4)(*self.dims)
        st = self._lib.ovd_create_lattice(dims_c, m0, r, t_bc, ctypes.byref(opt),
                                          ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != OVD_OK:
            raise OvdError(st, "ovd_create_lattice failed (check dims >= 2, r == 1, t_bc = +-1)")
        self._h = h

    # -- helpers --
    def _raise(self, st):
        msg = self._lib.ovd_last_error(self._h).decode()
        if st == OVD_EBREAKDOWN:
            raise Breakdown(st, msg)
        raise OvdError(st, msg)

    def _call(self, name, *args):
        st = getattr(self._lib, name)(self._h, *args)
        if st != OVD_OK:
            self._raise(st)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ovd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stats(s):
        return Stats(s.k, s.breakdown_step, s.min_margin, s.sign_check, s.ms_lanczos, s.ms_small_sign, s.ms_total,
                     s.ms_stencil, s.ms_update, s.basis_recomputed)

    def _dir(self, direction, dU):
        if direction in (None, "mu", DIR_MU):
            return _Dir(DIR_MU, None), None
        if dU is None:
            raise ValueError("link direction needs dU")
        _check_field(dU, (4, self.V, 3, 3), "dU")
        return _Dir(DIR_LINK, ctypes.c_void_p(dU.data_ptr())), dU

    # -- API --
    def set_links(self, U):
        _check_field(U, (4, self.V, 3, 3), "U")
        self._call("ovd_set_links", _ptr(U))
        self._U = U

    def apply_op(self, op, mu, inp, dU=None):
        """op in {OP_H, OP_DW, OP_DH_DMU, OP_DH_DLINK}; inp [n, V, 4, 3] complex128."""
        n = inp.shape[0]
        _check_field(inp, (n, self.V, 4, 3), "input")
        out = torch.empty_like(inp)
        d, keep = self._dir("link" if op == OP_DH_DLINK else None, dU)
        ms = ctypes.c_double(0.0)
        self._call("ovd_apply_op", op, float(mu), ctypes.byref(d), n, _ptr(inp), _ptr(out), ctypes.byref(ms))
        self.last_ms = ms.value
        return out

    def sign_apply(self, b, mu, k):
        """sgn(H(mu)) b by k steps of two-sided Lanczos; b [n, V, 4, 3]; mu scalar or list of n."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        y = torch.empty_like(b)
        st = _Stats()
        self._call("ovd_sign_apply", n, _dbl(mus), int(k), _ptr(b), _ptr(y), ctypes.byref(st))
        self.last_stats = self._stats(st)
        return y

    def sign_apply_deriv(self, b, mu, k, direction="mu", dU=None, want_vectors=True, x=None):
        """Derivative of sgn(H(mu)) b along mu or a link tangent dU (eq. 6-7).

        Returns (y, dy, xdy): y = sgn(H) b and dy = d/dt sgn(H) b when
        want_vectors, xdy = <x|dy> (one complex per source) when x is given;
        without want_vectors the Krylov basis is never stored."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        if x is not None:
            _check_field(x, (n, self.V, 4, 3), "x")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        d, keep = self._dir(direction, dU)
        y = torch.empty_like(b) if want_vectors else None
        dy = torch.empty_like(b) if want_vectors else None
        xdy = (ctypes.c_double * (2 * n))() if x is not None else None
        st = _Stats()
        self._call("ovd_sign_apply_deriv", n, _dbl(mus), ctypes.byref(d), int(k), _ptr(b), _ptr(y), _ptr(dy),
                   _ptr(x), xdy, ctypes.byref(st))
        self.last_stats = self._stats(st)
        s = None
        if xdy is not None:
            s = [complex(xdy[2 * i], xdy[2 * i + 1]) for i in range(n)]
        return y, dy, s

    def sign_apply_deriv_noalloc(self, b, x, mu, k, direction="mu", dU=None):
        """<x|d/dt sgn(H(mu)) b> per source like sign_apply_deriv in its
        storage-free mode, with no device allocation by the library (every
        workspace in its static per-device scratch; ovd_sign_apply_deriv_noalloc)."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        _check_field(x, (n, self.V, 4, 3), "x")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        d, keep = self._dir(direction, dU)
        xdy = (ctypes.c_double * (2 * n))()
        st = _Stats()
        self._call("ovd_sign_apply_deriv_noalloc", n, _dbl(mus), ctypes.byref(d), int(k), _ptr(b), _ptr(x), xdy,
                   ctypes.byref(st))
        self.last_stats = self._stats(st)
        return [complex(xdy[2 * i], xdy[2 * i + 1]) for i in range(n)]

    def overlap_apply(self, b, mu, k, deriv=False, direction="mu", dU=None):
        """D_ov b = b + gamma5 sgn(H) b (eq. 1, a = 1), and with deriv=True also
        d/dt D_ov b = gamma5 d/dt sgn(H) b.  Returns Db or (Db, dDb)."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        d, keep = self._dir(direction if deriv else None, dU)
        Db = torch.empty_like(b)
        dDb = torch.empty_like(b) if deriv else None
        st = _Stats()
        self._call("ovd_overlap_apply", n, _dbl(mus), ctypes.byref(d), int(k), _ptr(b), _ptr(Db), _ptr(dDb),
                   ctypes.byref(st))
        self.last_stats = self._stats(st)
        return (Db, dDb) if deriv else Db

    def sign_error_estimate(self, b, mu, k):
        """Sec. 4 estimate |sgn(H)^2 b - b| / (2 |b|) per source (k steps, applied twice)."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        eps = (ctypes.c_double * n)()
        st = _Stats()
        self._call("ovd_sign_error_estimate", n, _dbl(mus), int(k), _ptr(b), eps, ctypes.byref(st))
        return [eps[i] for i in range(n)]

    def block_sign_apply(self, t, b, mu, k, direction="mu", dU=None):
        """sgn(B) (t; b) for the block matrix of eq. 6 (t may be None: zero top
        half).  Returns (yt, yb), the top and bottom halves."""
        n = b.shape[0]
        _check_field(b, (n, self.V, 4, 3), "b")
        if t is not None:
            _check_field(t, (n, self.V, 4, 3), "t")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        d, keep = self._dir(direction, dU)
        yt, yb = torch.empty_like(b), torch.empty_like(b)
        st = _Stats()
        self._call("ovd_block_sign_apply", n, _dbl(mus), ctypes.byref(d), int(k), _ptr(t), _ptr(b), _ptr(yt),
                   _ptr(yb), ctypes.byref(st))
        self.last_stats = self._stats(st)
        return yt, yb

    def deriv_error_estimate(self, phi, mu, k, direction="mu", dU=None):
        """Sec. 4 estimate for the derivative: |sgn(B)^2 (0; phi) - (0; phi)| / (2 |phi|) per source."""
        n = phi.shape[0]
        _check_field(phi, (n, self.V, 4, 3), "phi")
        mus = [float(mu)] * n if not hasattr(mu, "__len__") else [float(m) for m in mu]
        d, keep = self._dir(direction, dU)
        eps = (ctypes.c_double * n)()
        st = _Stats()
        self._call("ovd_deriv_error_estimate", n, _dbl(mus), ctypes.byref(d), int(k), _ptr(phi), eps,
                   ctypes.byref(st))
        return [eps[i] for i in range(n)]

    def sign_apply_vjp(self, x, b, mu, k, force=True, wirtinger=False, grad=True, u1=False):
        """s = <x|sgn(H(mu))|b>, ds/dmu and the link gradients (FP64 results;
        the Lanczos run in the handle's precision).

        Returns (s, ds_dmu, F, dsdU, dsdUc); F = per-link force [4, V, 3, 3]
        (ds/dt = tr(F X) for U -> e^{tX} U) when force, and the Wirtinger
        derivatives ds/dU, ds/dconj(U) when wirtinger.  With grad=False only s
        is computed (ds_dmu is None).  The handle's basis_recompute chooses
        between keeping both Krylov bases and regenerating the right one
        (last_stats.basis_recomputed tells which ran).  With u1=True the U(1)
        derivatives ds/dTheta_nu(y) = i tr F_nu(y) ([4, V] complex) are stored
        in self.last_dsdtheta."""
        _check_field(x, (1, self.V, 4, 3), "x")
        _check_field(b, (1, self.V, 4, 3), "b")
        sc = (ctypes.c_double * 2)()
        dm = (ctypes.c_double * 2)() if grad else None
        opts = dict(dtype=torch.complex128, device=b.device)
        F = torch.empty((4, self.V, 3, 3), **opts) if grad and force else None
        dU = torch.empty((4, self.V, 3, 3), **opts) if grad and wirtinger else None
        dUc = torch.empty((4, self.V, 3, 3), **opts) if grad and wirtinger else None
        dth = torch.empty((4, self.V), **opts) if grad and u1 else None
        st = _Stats()
        self._call("ovd_sign_apply_vjp", float(mu), int(k), _ptr(x), _ptr(b), sc, dm, _ptr(F), _ptr(dU), _ptr(dUc),
                   _ptr(dth), ctypes.byref(st))
        self.last_dsdtheta = dth
        self.last_stats = self._stats(st)
        return complex(sc[0], sc[1]), (complex(dm[0], dm[1]) if grad else None), F, dU, dUc

    def set_deflation(self, mu, lam, R, L, l=0, dR=None, dL=None, direction="mu", dU=None):
        """Deflation set for one mu (eq. 8 with the m pairs, eq. 11 with the first l).

        lam: m complex eigenvalues (closest to zero first); R, L: [m, V, 4, 3]
        right / left eigenvectors with L^dag R = 1; dR, dL: [l, V, 4, 3]
        derivatives of the first l along `direction`."""
        m = len(lam)
        _check_field(R, (m, self.V, 4, 3), "R")
        _check_field(L, (m, self.V, 4, 3), "L")
        if l > 0:
            _check_field(dR, (l, self.V, 4, 3), "dR")
            _check_field(dL, (l, self.V, 4, 3), "dL")
        lam_c = (ctypes.c_double * (2 * m))()
        for i, z in enumerate(lam):
            lam_c[2 * i] = float(complex(z).real)
            lam_c[2 * i + 1] = float(complex(z).imag)
        link = direction in ("link", DIR_LINK)
        if link and l > 0 and dU is not None:
            _check_field(dU, (4, self.V, 3, 3), "dU")
        d = _Dir(DIR_LINK if link else DIR_MU, ctypes.c_void_p(dU.data_ptr()) if link and dU is not None else None)
        self._call("ovd_set_deflation", float(mu), m, lam_c, _ptr(R), _ptr(L), int(l),
                   _ptr(dR) if l > 0 else None, _ptr(dL) if l > 0 else None, ctypes.byref(d))

    def compute_deflation(self, mu, m, l=0, direction="mu", dU=None, tol=1e-10):
        """Eigenpairs of smallest |lambda| (and derivatives of the first l) on the
        GPU, installed as the deflation set of mu.  Returns (lam, stats)."""
        dirs, keep = self._dir(direction if l > 0 else None, dU)
        lam = (ctypes.c_double * (2 * m))()
        st = _EigStats()
        self._call("ovd_compute_deflation", float(mu), int(m), int(l), ctypes.byref(dirs), float(tol), lam,
                   ctypes.byref(st))
        import numpy as np
        lv = np.array([complex(lam[2 * i], lam[2 * i + 1]) for i in range(m)])
        stats = {f: getattr(st, f) for f, _ in _EigStats._fields_}
        return lv, stats

    def tuned_shapes(self):
        """Launch shapes chosen by the autotuner so far (see ovd_get_tuned)."""
        buf = ctypes.create_string_buffer(4096)
        self._call("ovd_get_tuned", buf, 4096)
        return buf.value.decode()

    def get_deflation(self, mu):
        """(lam, R, L, dR, dL) of the deflation set of mu; dR, dL None if l = 0."""
        m, l = ctypes.c_int(0), ctypes.c_int(0)
        self._call("ovd_get_deflation", float(mu), ctypes.byref(m), ctypes.byref(l), None, None, None, None, None)
        m, l = m.value, l.value
        lam = (ctypes.c_double * (2 * m))()
        opts = dict(dtype=torch.complex128, device="cuda")
        R = torch.empty((m, self.V, 4, 3), **opts)
        L = torch.empty((m, self.V, 4, 3), **opts)
        dR = torch.empty((l, self.V, 4, 3), **opts) if l > 0 else None
        dL = torch.empty((l, self.V, 4, 3), **opts) if l > 0 else None
        self._call("ovd_get_deflation", float(mu), None, None, lam, _ptr(R), _ptr(L), _ptr(dR), _ptr(dL))
        import numpy as np
        lv = np.array([complex(lam[2 * i], lam[2 * i + 1]) for i in range(m)])
        return lv, R, L, dR, dL

    def clear_deflation(self):
        self._call("ovd_clear_deflation")

    def get_tridiag(self, k, rhs=0):
        """(alpha, beta, delta) of the last Lanczos run as lists of complex."""
        a = (ctypes.c_double * (2 * k))()
        b = (ctypes.c_double * (2 * k))()
        d = (ctypes.c_double * (2 * k))()
        self._call("ovd_get_tridiag", int(rhs), int(k), a, b, d)
        cv = lambda arr: [complex(arr[2 * i], arr[2 * i + 1]) for i in range(k)]
        return cv(a), cv(b), cv(d)


def sign_apply_deriv_batch(jobs):
    """Uneven batch: jobs = [(lattice, b, mu, k, x), ...] or, for a link
    direction, [(lattice, b, mu, k, x, dU), ...], one per lattice (distinct
    handles, ideally created on distinct streams); every lattice's derivative
    <x|d/dt sgn(H) b> (ovd_sign_apply_deriv_batch).  Lattices of one precision
    and one kind of direction share one update and one stencil launch per
    Lanczos step unless a handle was created with batch_separate=True.
    Returns a list of per-lattice lists of complex values."""
    n = len(jobs)
    arr = (_Job * n)()
    keep = []
    outs = []
    for i, job in enumerate(jobs):
        lat, b, mu, k, x = job[:5]
        dU = job[5] if len(job) > 5 else None
        nr = b.shape[0]
        _check_field(b, (nr, lat.V, 4, 3), "b")
        _check_field(x, (nr, lat.V, 4, 3), "x")
        mus = [float(mu)] * nr if not hasattr(mu, "__len__") else [float(m) for m in mu]
        mu_c = _dbl(mus)
        xdy = (ctypes.c_double * (2 * nr))()
        st = _Stats()
        d, kd = lat._dir("link" if dU is not None else None, dU)
        keep += [mu_c, xdy, st, b, x, d, kd]
        arr[i] = _Job(lat._h.value if hasattr(lat._h, "value") else lat._h, nr,
                      ctypes.cast(mu_c, ctypes.POINTER(ctypes.c_double)), ctypes.addressof(d), int(k), b.data_ptr(),
                      None, None, x.data_ptr(), ctypes.cast(xdy, ctypes.POINTER(ctypes.c_double)),
                      ctypes.pointer(st), 0)
        outs.append((xdy, nr, lat, st))
    status = lib().ovd_sign_apply_deriv_batch(n, arr)
    if status != OVD_OK:
        for i in range(n):
            if arr[i].status != OVD_OK:
                outs[i][2]._raise(arr[i].status)
        raise OvdError(status, "ovd_sign_apply_deriv_batch failed")
    res = []
    for xdy, nr, lat, st in outs:
        lat.last_stats = Lattice._stats(st)
        res.append([complex(xdy[2 * j], xdy[2 * j + 1]) for j in range(nr)])
    return res


def tridiag_sign(alpha, beta, delta, method=SIGN_QUAD, quad_step=0.1, quad_max_levels=0, nested_inner=0,
                 breakdown_tol=1e-14):
    """sgn(T) e_1 for complex tridiagonal matrices given as numpy arrays
    [nt, k] (ovd_tridiag_sign; the ovd_get_tridiag convention: T[i][i+1] =
    beta[i+1], T[i+1][i] = delta[i+1]).  Returns (c [nt, k], check); raises
    OvdError with status OVD_ENOCONV when the quadrature levels run out."""
    import numpy as np
    a = np.ascontiguousarray(np.atleast_2d(alpha), dtype=np.complex128)
    b = np.ascontiguousarray(np.atleast_2d(beta), dtype=np.complex128)
    d = np.ascontiguousarray(np.atleast_2d(delta), dtype=np.complex128)
    nt, k = a.shape
    if b.shape != a.shape or d.shape != a.shape:
        raise ValueError("alpha, beta, delta must have the same shape [nt, k]")
    opt = _Options(FP64, LEFT_SUM, breakdown_tol, quad_step, 0, 1, 1, -1, 0, -1, 0, -1, int(quad_max_levels),
                   int(method), int(nested_inner), 0, 0)
    c = np.zeros((nt, k), dtype=np.complex128)
    chk = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib().ovd_tridiag_sign(nt, k, a.ctypes.data_as(dp), b.ctypes.data_as(dp), d.ctypes.data_as(dp),
                                ctypes.byref(opt), c.ctypes.data_as(dp), ctypes.byref(chk),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != OVD_OK:
        err = OvdError(st, "ovd_tridiag_sign failed")
        err.check = chk.value
        err.c = c
        raise err
    return c, chk.value


def create_lattice(dims, **kw) -> Lattice:
    return Lattice(dims, **kw)
