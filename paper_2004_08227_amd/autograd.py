"""PyTorch autograd wrapper of the MPLP++ adjoint.

``mplp_dual(unaries, pairwise, edges, K, every)`` runs K MPLP++ iterations
from phi = 0 on the GPU and returns D_K = sum_u min_s U_u(s), the dual bound
of Eq. (3) after K sweeps; its backward calls the library's hand-written
adjoint (argmin-selection subgradients, checkpoints every `every` iterations),
so unary and pairwise potentials can be learned.  Torch provides only the
device memory of inputs and gradients.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Solver


class MPLPDual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, unaries, pairwise, edges, K, every):
        n, L = unaries.shape
        un = unaries.detach().contiguous()
        pw = pairwise.detach().contiguous()
        torch.cuda.current_stream().synchronize()
        solver = Solver.from_torch(n, L, np.asarray(edges, dtype=np.int32), un, pw)
        loss = solver.adjoint_forward(int(K), int(every))
        ctx.solver = solver
        ctx.meta = (unaries.shape, pairwise.shape, unaries.dtype, unaries.device)
        return torch.tensor(loss, dtype=unaries.dtype, device=unaries.device)

    @staticmethod
    def backward(ctx, grad_out):
        ushape, pshape, dtype, device = ctx.meta
        gu = torch.empty(ushape, dtype=dtype, device=device)
        gp = torch.empty(pshape, dtype=dtype, device=device)
        torch.cuda.current_stream().synchronize()
        ctx.solver.adjoint_backward_device(gu, gp)
        ctx.solver.close()
        ctx.solver = None
        return grad_out * gu, grad_out * gp, None, None, None


def mplp_dual(unaries, pairwise, edges, K=50, every=10):
    """D_K of the model (unaries [n, L], pairwise [m, L, L] on the GPU, edges
    int32 [m, 2] on the host), differentiable with respect to both tensors."""
    return MPLPDual.apply(unaries, pairwise, edges, K, every)
