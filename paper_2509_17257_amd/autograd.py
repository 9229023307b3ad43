"""torch.autograd wrappers of the H^2 product and of the block-CG solve.

Every forward and backward step is a call into libh2x.so (products, adjoint
products, gradient kernels, block CG); this module only wires them into
autograd.

``h2_apply(A, X, ell=None, coupling=None)``  ->  Y = A X
    backward: dX = A^T dY (adjoint product through the column lists),
    d ell = sum over admissible blocks of <dS_b/d ell, dyhat_t xhat_s^T> plus the
    near-field term (h2x_grad; the near-field term alone when ``coupling`` is given,
    since the supplied coupling matrices do not depend on ell), and the gradient of
    the coupling matrices dS_b = dyhat_t xhat_s^T.

``h2_solve(A, B, ell=None, coupling=None, rtol=...)``  ->  X = A^{-1} B (block CG)
    backward (implicit adjoint): Lambda = A^{-T} dX by block CG (the H^2
    approximation is exactly symmetric: S_(s,t) = S_(t,s)^T and N_(s,t) = N_(t,s)^T
    because the kernel is symmetric and both blocks use the same interpolation
    nodes), dB = Lambda, and the operator gradients of <dX, X> are minus those of
    <Lambda, A X>: dS_b = -lambdahat_t xhat_s^T, d ell = -<Lambda, (dA/d ell) X>.

``ell`` is an optional 0-d float64 tensor: the operator is refilled at that
length scale before the forward step when it differs from the current one, and
receives d L / d ell.  ``coupling`` is an optional (n_adm, k, k) float64 CUDA
tensor of coupling matrices in the block order of ``Plan.blocks()`` (start from
``A.coupling()``): it is uploaded into the operator before the forward step and
receives d L / d S.  The operator must not be changed between a forward step
and its backward step.
"""
from __future__ import annotations

import torch

from . import H2Matrix, H2xError, block_cg_solve, h2_grad, h2_matmul, h2_matmul_adjoint

__all__ = ["h2_apply", "h2_solve"]


def _sync(A: H2Matrix, ell, coupling):
    if ell is not None:
        v = float(ell.detach().cpu())
        if v != A.ell:
            A.set_ell(v)
    if coupling is not None:
        A.set_coupling(coupling.detach())


def _operator_grads(ctx, A, X, W, sign):
    """Gradients of sign * <W, A X> w.r.t. ell and the coupling matrices.  When the coupling
    matrices are supplied by the caller they do not depend on ell: d ell is then the
    near-field term alone."""
    want_ell = ctx.needs_input_grad[1]
    want_S = ctx.needs_input_grad[2]
    if not (want_ell or want_S):
        return None, None
    terms = "near" if ctx.S_device is not None else "all"
    dS, _, dl = h2_grad(A, X, W, want_dS=want_S, want_dN=False, want_dell=want_ell, scale=sign, dell_terms=terms)
    if dl is not None:
        dl = dl.to(ctx.ell_device).reshape(ctx.ell_shape)
    if dS is not None and dS.device != ctx.S_device:
        dS = dS.to(ctx.S_device)
    return dl, dS


class _Apply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, ell, coupling, A):
        _sync(A, ell, coupling)
        X = X.contiguous()
        ctx.A = A
        ctx.ell_device, ctx.ell_shape = (ell.device, ell.shape) if ell is not None else (None, None)
        ctx.S_device = coupling.device if coupling is not None else None
        ctx.save_for_backward(X)
        return h2_matmul(A, X)

    @staticmethod
    def backward(ctx, dY):
        A = ctx.A
        (X,) = ctx.saved_tensors
        dY = dY.contiguous()
        dX = h2_matmul_adjoint(A, dY) if ctx.needs_input_grad[0] else None
        dl, dS = _operator_grads(ctx, A, X, dY, 1.0)
        return dX, dl, dS, None


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, ell, coupling, A, opts):
        _sync(A, ell, coupling)
        B = B.contiguous()
        X, info = block_cg_solve(A, B, **opts)
        if info.status != 0:
            raise H2xError(f"h2_solve: block CG ended with status {info.status} after {info.iters} iterations")
        ctx.A, ctx.opts = A, opts
        ctx.ell_device, ctx.ell_shape = (ell.device, ell.shape) if ell is not None else (None, None)
        ctx.S_device = coupling.device if coupling is not None else None
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, dX):
        A = ctx.A
        (X,) = ctx.saved_tensors
        lam, info = block_cg_solve(A, dX.contiguous(), **ctx.opts)
        if info.status != 0:
            raise H2xError(f"h2_solve backward: block CG ended with status {info.status}")
        dl, dS = _operator_grads(ctx, A, X, lam, -1.0)
        return (lam if ctx.needs_input_grad[0] else None), dl, dS, None, None


def h2_apply(A: H2Matrix, X, ell=None, coupling=None):
    """Y = A X with autograd support for X, ell and the coupling matrices."""
    return _Apply.apply(X, ell, coupling, A)


def h2_solve(A: H2Matrix, B, ell=None, coupling=None, *, rtol=1e-10, max_iter=10000, variant="independent"):
    """X = A^{-1} B by block CG, with the implicit-adjoint backward."""
    return _Solve.apply(B, ell, coupling, A, dict(rtol=rtol, max_iter=max_iter, variant=variant))
