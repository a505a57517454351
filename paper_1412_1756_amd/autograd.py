"""torch.autograd face of the MLFMA product (argument marshalling only: the
forward, the adjoint pass, the dZ/dk pass and the gradient reduction all run
in the library).

y = Z(k) x.  Backward with PyTorch's complex convention:
  x_bar = Z^H y_bar                    (adjoint pass: conjugated input/output, Z = Z^T)
  k_bar = Re( sum conj(y_bar) * (dZ/dk x) )   (dual-number pass, tree and sampling
                                               frozen; the sum by cm_vdot)
"""
import torch


class ZApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, k, op):
        ctx.op = op
        ctx.save_for_backward(x)
        return op.apply(x, "Z")

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        op = ctx.op
        gx = gk = None
        g = g.contiguous()
        if ctx.needs_input_grad[0]:
            gx = op.apply(g, "ZH")
        if ctx.needs_input_grad[1]:
            dzx = op.apply(x, "DZDK")
            gk = op.vdot(g, dzx).real
        return gx, gk, None


def z_apply(op, x, k):
    """Differentiable y = Z(k) x; k is a real scalar tensor standing for the
    wavenumber the operator was built at (its value is not re-read)."""
    return ZApply.apply(x, k, op)


def dlambda_dk(op, lam, X):
    """Derivatives d lambda/dk of one characteristic value (or one degenerate
    cluster) from its Ritz vectors X ((N,) or (N, m) CUDA complex128 tensor):

      d lambda/dk = eig( Q^T (X' - lambda R') Q ),  Q^T R Q = I,

    with Q a real R-orthonormal basis of the cluster's span (real and
    imaginary parts of the Ritz vectors), X' = Im dZ/dk and R' = Re dZ/dk
    (cm_dlambda_dk; lam: the value, or the cluster's values, whose real mean
    is taken).  For a single mode this is J^T (X' - lambda R') J / J^T R J.
    Returns a sorted numpy array of m derivatives."""
    import numpy as np
    lam_r = float(np.real(np.mean(np.atleast_1d(lam))))
    return op.dlambda_dk(lam_r, X)
