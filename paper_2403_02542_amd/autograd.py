"""torch.autograd bindings of the hand-written adjoints.

`local_energy(ctx, sys_id, h, L)` returns Re E_L of every walker of a system
(Eq. eloc) as a float64 tensor whose backward runs afq_local_energy_adjoint;
`coulomb_vector(ctx, sys_id, L)` returns the Coulomb vector ell_g = 2 tr T_g
(complex128, [W][n_chol], the input of the force bias of Eq. force_shift)
with backward afq_force_bias_adjoint.  Both differentiate at fixed walkers
and fixed Psi_T with respect to the unconstrained entries of h and L_g.

h and L must be the very tensors the system was built from (checked by
storage address and version), so that the gradient belongs to the values the
library holds.  Both sides of every call synchronise the context stream with
torch's current stream.
"""
from __future__ import annotations

import torch

from . import afq


def _check_source(ctx: afq.Context, sys_id: int, h, L):
    src = ctx.dims[sys_id].get("src")
    now = (None if h is None else (h.data_ptr(), h._version), (L.data_ptr(), L._version))
    if src is None or (h is not None and src[0] != now[0]) or src[1] != now[1]:
        raise ValueError("h / L are not the device tensors this system was built from "
                         "(or were modified since)")


class _LocalEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, h, L, ctx, sys_id, precision):
        d = ctx.dims[sys_id]
        e = torch.empty(d["W"], dtype=torch.complex128, device=h.device)
        torch.cuda.current_stream().synchronize()
        ctx.local_energy_batch(sys_id, eloc_out=e, precision=precision)
        ctx.sync()
        fctx.afq = (ctx, sys_id)
        return e.real.contiguous()

    @staticmethod
    def backward(fctx, grad):
        ctx, sys_id = fctx.afq
        d = ctx.dims[sys_id]
        M, G = d["M"], d["G"]
        gh = torch.empty((M, M), dtype=torch.float64, device=grad.device)
        gL = torch.empty((G, M, M), dtype=torch.float64, device=grad.device)
        g = grad.to(torch.float64).contiguous()
        torch.cuda.current_stream().synchronize()
        ctx.local_energy_adjoint(sys_id, g, gh, gL)
        ctx.sync()
        return gh, gL, None, None, None


class _CoulombVector(torch.autograd.Function):
    @staticmethod
    def forward(fctx, L, ctx, sys_id):
        d = ctx.dims[sys_id]
        e = torch.empty(d["W"], dtype=torch.complex128, device=L.device)
        ell = torch.empty((d["W"], d["G"]), dtype=torch.complex128, device=L.device)
        torch.cuda.current_stream().synchronize()
        ctx.local_energy_batch(sys_id, eloc_out=e, ell_out=ell)
        ctx.sync()
        fctx.afq = (ctx, sys_id)
        return ell

    @staticmethod
    def backward(fctx, grad):
        # For a real loss, torch hands over dl/dRe(ell) + i dl/dIm(ell).
        ctx, sys_id = fctx.afq
        d = ctx.dims[sys_id]
        M, G = d["M"], d["G"]
        gL = torch.empty((G, M, M), dtype=torch.float64, device=grad.device)
        g = grad.to(torch.complex128).contiguous()
        torch.cuda.current_stream().synchronize()
        ctx.force_bias_adjoint(sys_id, g, gL)
        ctx.sync()
        return gL, None, None


def local_energy(ctx: afq.Context, sys_id: int, h: torch.Tensor, L: torch.Tensor,
                 precision: int = afq.PREC_FP64) -> torch.Tensor:
    """Re E_L [W] with gradients to h [M][M] and L [n_chol][M][M]."""
    _check_source(ctx, sys_id, h, L)
    return _LocalEnergy.apply(h, L, ctx, sys_id, precision)


def coulomb_vector(ctx: afq.Context, sys_id: int, L: torch.Tensor) -> torch.Tensor:
    """ell [W][n_chol] complex with gradients to L [n_chol][M][M]."""
    _check_source(ctx, sys_id, None, L)
    return _CoulombVector.apply(L, ctx, sys_id)
