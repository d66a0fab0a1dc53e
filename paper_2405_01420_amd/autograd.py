"""torch.autograd.Function over the C-ABI: forces and energies forward, the hand-written adjoint
kernel backward.  Torch supplies device memory and the current stream only; every step of the
computation runs in libnb's kernels.

    F, E_LJ, E_C = NonbondedFunction.apply(x, q, sigma, epsilon, types, ctx)

x [N, 3] float32 (cuda), q [N] float32, sigma / epsilon [ntypes] float64, types [N] int32,
ctx a context from nb.nb_setup.  The forward rebuilds the pair list from x; the backward
rebuilds it again from the saved x (no per-pair tape is stored) and calls nb_backward, which
returns dL/dx (a Hessian-vector product plus the energy term), dL/dq, dL/dsigma, dL/deps.
"""
from __future__ import annotations

import torch

from . import nb


class NonbondedFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, q, sigma, epsilon, types, nbctx):
        xc = x.detach().contiguous()
        qc = q.detach().contiguous()
        tc = types.contiguous()
        nb.nb_set_lj(nbctx, sigma.detach().double().cpu().numpy(), epsilon.detach().double().cpu().numpy())
        nb.nb_pairlist(nbctx, xc)
        f = torch.empty_like(xc)
        e = torch.empty(2, dtype=torch.float64, device=xc.device)
        nb.nb_forces(nbctx, xc, qc, tc, f, e)
        ctx.save_for_backward(xc, qc, tc, sigma, epsilon)
        ctx.nbctx = nbctx
        return f, e[0], e[1]

    @staticmethod
    def backward(ctx, gf, ge_lj, ge_c):
        x, q, types, sigma, epsilon = ctx.saved_tensors
        nbctx = ctx.nbctx
        dev = x.device
        gf = torch.zeros_like(x) if gf is None else gf.contiguous().float()
        ge = torch.stack([torch.zeros((), dtype=torch.float64, device=dev) if ge_lj is None else ge_lj.double(),
                          torch.zeros((), dtype=torch.float64, device=dev) if ge_c is None else ge_c.double()]).contiguous()
        dx = torch.empty_like(x)
        dq = torch.empty_like(q)
        dsig = torch.empty(sigma.shape[0], dtype=torch.float64, device=dev)
        deps = torch.empty(epsilon.shape[0], dtype=torch.float64, device=dev)
        nb.nb_set_lj(nbctx, sigma.detach().double().cpu().numpy(), epsilon.detach().double().cpu().numpy())
        nb.nb_backward(nbctx, x, q, types, gf, ge, dx, dq, dsig, deps, 0)
        return dx, dq, dsig.to(sigma.dtype), deps.to(epsilon.dtype), None, None


def nonbonded(x, q, sigma, epsilon, types, nbctx):
    """Convenience wrapper: returns (F [N,3], E_LJ, E_C) with autograd support."""
    return NonbondedFunction.apply(x, q, sigma, epsilon, types, nbctx)
