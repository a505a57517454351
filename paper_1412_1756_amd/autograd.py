"""torch.autograd face of the MLFMA product (argument marshalling only: the
forward, the adjoint pass and the dZ/dk pass all run in the library).

y = Z(k) x.  Backward with PyTorch's complex convention:
  x_bar = Z^H y_bar                    (adjoint pass: conjugated input/output, Z = Z^T)
  k_bar = Re( sum conj(y_bar) * (dZ/dk x) )   (dual-number pass, tree and sampling frozen)
"""
import numpy as np
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
            gk = (torch.conj(g) * dzx).real.sum().to(torch.float64)
        return gx, gk, None


def z_apply(op, x, k):
    """Differentiable y = Z(k) x; k is a real scalar tensor standing for the
    wavenumber the operator was built at (its value is not re-read)."""
    return ZApply.apply(x, k, op)


def dlambda_dk(op, lam, X):
    """Derivatives d lambda/dk of one characteristic value (or one degenerate
    cluster) from its Ritz vectors X (N x m CUDA tensor):

      d lambda/dk = eig( Q^T (X' - lambda R') Q ),  Q^T R Q = I,

    with Q a real R-orthonormal basis of the cluster's span (real and
    imaginary parts of the Ritz vectors), X' = Im dZ/dk and R' = Re dZ/dk.
    For a single mode this is J^T (X' - lambda R') J / J^T R J.  Returns a
    sorted numpy array of m derivatives."""
    if X.dim() == 1:
        X = X.reshape(-1, 1)
    m = X.shape[1]
    Xh = X.detach().cpu().numpy()
    W = np.ascontiguousarray(np.concatenate([Xh.real, Xh.imag], axis=1))     # N x 2m, real span
    dev = X.device
    RW = op.apply(torch.tensor(W, dtype=torch.complex128, device=dev), "R").cpu().numpy().real
    # small dense projections on the host (m is the cluster size)
    Gm = W.T @ RW
    Gm = 0.5 * (Gm + Gm.T)
    ev, U = np.linalg.eigh(Gm)
    keep = np.argsort(ev)[::-1][:m]
    Q = W @ (U[:, keep] / np.sqrt(ev[keep])[None, :])                        # N x m, Q^T R Q = I
    D = op.apply(torch.tensor(Q, dtype=torch.complex128, device=dev), "DZDK").cpu().numpy()
    lam_r = float(np.real(np.mean(lam)))
    M = Q.T @ (D.imag - lam_r * D.real)
    return np.sort(np.linalg.eigvalsh(0.5 * (M + M.T)))
