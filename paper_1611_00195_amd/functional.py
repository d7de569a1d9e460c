"""Differentiable s = <x|sgn(H(mu))|b> for PyTorch autograd, on the library's VJP.

The bilinear <x|sgn(H)|b> is the quantity whose derivatives give the
conserved currents and the fermionic force the paper's derivatives serve
(Sec. 1).  ``sign_bilinear`` returns it as a complex 0-dim tensor whose
backward pass calls ``ovd_sign_apply_vjp``: one two-sided Lanczos run with
both Krylov bases kept, M_k = L_sgn(T_k, e_1 e_1^T) for the Frechet derivative
of the sign function (eq. 6 applied to T_k), and one per-link contraction for
all links at once -- no per-direction derivative runs.

PyTorch's complex convention: for a real loss L and incoming gradient g of
s, the gradient of a complex input z is conj(g) ds/dconj(z) + g conj(ds/dz),
and of the real mu it is Re(conj(g) ds/dmu).  The links are treated as
unconstrained complex 3x3 matrices (Wirtinger derivatives); the gradients of
x and b need one more sign application each: ds/dconj(x) = sgn(H) b and
ds/db = (sgn(H)^dag x)^T with sgn(H)^dag = sgn(H(-mu)).
"""
from __future__ import annotations

import torch

from .ovderiv import Lattice


def _as_field(t, V):
    return t.reshape(1, V, 4, 3).contiguous()


class SignBilinear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, mu, x, b, lat: Lattice, k: int):
        V = lat.V
        need_U, need_mu, need_x, need_b = ctx.needs_input_grad[:4]
        Uc = U.detach().contiguous()
        lat.set_links(Uc)
        xf = _as_field(x.detach(), V)
        bf = _as_field(b.detach(), V)
        grad = need_U or need_mu
        s, dsdmu, _, dU, dUc = lat.sign_apply_vjp(xf, bf, float(mu), k, force=False, wirtinger=need_U, grad=grad)
        ctx.lat, ctx.k, ctx.mu = lat, k, float(mu)
        ctx.mu_meta = (mu.device, mu.dtype)
        ctx.dsdmu = dsdmu
        ctx.save_for_backward(Uc, xf, bf, dU, dUc)
        ctx.x_shape, ctx.b_shape = x.shape, b.shape
        return torch.tensor(s, dtype=torch.complex128, device=b.device)

    @staticmethod
    def backward(ctx, g):
        Uc, xf, bf, dU, dUc = ctx.saved_tensors
        need_U, need_mu, need_x, need_b = ctx.needs_input_grad[:4]
        gU = gmu = gx = gb = None
        if need_U:
            gU = torch.conj(g) * dUc + g * torch.conj(dU)
        if need_mu:
            gmu = (torch.conj(g) * ctx.dsdmu).real.to(device=ctx.mu_meta[0], dtype=ctx.mu_meta[1])
        if need_x or need_b:
            lat = ctx.lat
            lat.set_links(Uc)
            if need_x:   # s is antilinear in x: ds/dconj(x) = sgn(H) b
                gx = (torch.conj(g) * lat.sign_apply(bf, ctx.mu, ctx.k)).reshape(ctx.x_shape)
            if need_b:   # s is linear in b: conj(ds/db) = sgn(H(-mu)) x
                gb = (g * lat.sign_apply(xf, -ctx.mu, ctx.k)).reshape(ctx.b_shape)
        return gU, gmu, gx, gb, None, None


def sign_bilinear(lat: Lattice, U, mu, x, b, k: int):
    """s = <x|sgn(H(mu))|b> (complex128 0-dim tensor), differentiable in U, mu, x and b.

    U: complex128 [4, V, 3, 3] on the device; mu: float or 0-dim float64 tensor;
    x, b: complex128 with V*12 elements ([V, 4, 3] site-spin-colour order);
    k: Krylov dimension.  The lattice handle's links are overwritten with U,
    which removes its deflation sets (they belong to other links): the value
    and all four gradients come from undeflated runs of the same k."""
    if not isinstance(mu, torch.Tensor):
        mu = torch.tensor(float(mu), dtype=torch.float64)
    return SignBilinear.apply(U, mu, x, b, lat, int(k))
