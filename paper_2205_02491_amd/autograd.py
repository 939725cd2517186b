"""torch.autograd wrappers around the library's hand-written adjoints.

- ``chase_eigh(H, nev, nex, ...)``: eigenvalues and eigenvectors are
  differentiable.  Eigenvalues: dL/dH = V diag(dL/dlambda) V^H (first-order
  perturbation of a simple eigenvalue, ``chase_eigval_adjoint``).
  Eigenvectors, for losses that do not depend on the vectors' phases:
  ``chase_eigvec_adjoint`` (within-block divided differences plus
  conjugate-gradient solves on the complement of the eigenvectors).
- ``filtered_block(H, X0, degrees, b_sup, mu_1, mu_ne)``: the Chebyshev
  filter of X0 with the bounds and degrees held fixed; the backward replays
  the recurrence in reverse from the recorded intermediate blocks
  (``chase_filter_adjoint``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import (Handle, chase_eigval_adjoint, chase_eigvec_adjoint, chase_filter,
               chase_filter_adjoint, chase_solve, default_opts)


class ChaseEigh(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, nev, nex, tol, degree, V0, S, opts, adj_tol):
        ev, vec, res, st = chase_solve(H.detach(), nev, nex, tol, degree, V0, S, opts)
        vec = vec.contiguous()
        ctx.save_for_backward(H, vec)
        ctx.nev, ctx.nex, ctx.ev, ctx.adj_tol = nev, nex, ev, adj_tol
        lam = torch.tensor(ev, dtype=torch.float64, device=H.device)
        return lam, vec

    @staticmethod
    def backward(ctx, g_lam, g_vec):
        H, vec = ctx.saved_tensors
        n = vec.shape[0]
        dH = torch.zeros((n, n), dtype=vec.dtype, device=vec.device)
        if g_lam is not None:
            g = g_lam.detach().to(torch.float64).cpu().numpy()
            chase_eigval_adjoint(vec, g, dH)
        if g_vec is not None and bool(torch.any(g_vec != 0)):
            h = Handle(n, ctx.nev, ctx.nex, vec.dtype)
            try:
                chase_eigvec_adjoint(H.detach(), vec, ctx.ev, g_vec.detach().contiguous(), dH,
                                     handle=h, tol=ctx.adj_tol)
            finally:
                h.close()
        return dH, None, None, None, None, None, None, None, None


def chase_eigh(H, nev, nex, tol=1e-10, degree=20, V0=None, S=None, opts=None, adj_tol=1e-10):
    """Lowest nev eigenpairs (ascending eigenvalues, eigenvectors as columns)
    of the Hermitian H, differentiable w.r.t. H.  adj_tol: relative residual
    of the conjugate-gradient solves of the eigenvector adjoint."""
    return ChaseEigh.apply(H, nev, nex, tol, degree, V0, S, opts, adj_tol)


class FilteredBlock(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, X0, degrees, b_sup, mu_1, mu_ne):
        n, k = X0.shape
        h = Handle(n, max(1, k - 1) if k > 1 else 1, 1, H.dtype, default_opts())
        Y, _ = chase_filter(H.detach(), X0.detach(), degrees, b_sup, mu_1, mu_ne,
                            record_tape=True, handle=h)
        ctx.handle = h
        ctx.save_for_backward(H)
        return Y.contiguous()

    @staticmethod
    def backward(ctx, gY):
        (H,) = ctx.saved_tensors
        n = H.shape[0]
        dH = torch.zeros((n, n), dtype=H.dtype, device=H.device)
        gX = chase_filter_adjoint(H.detach(), gY.contiguous(), dH, ctx.handle,
                                  want_gX=ctx.needs_input_grad[1])
        ctx.handle.close()
        return dH, gX, None, None, None, None


def filtered_block(H, X0, degrees, b_sup, mu_1, mu_ne):
    degrees = np.asarray(degrees, dtype=np.int32)
    return FilteredBlock.apply(H, X0, degrees, b_sup, mu_1, mu_ne)
