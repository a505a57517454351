"""Sparse approximate inverse (SAI) of the near-field matrix (section IV).

The paper builds P with a prescribed sparsity pattern by minimising
||I - Z_near P||_F, which splits into one least-squares problem per column of
P, and names three thresholds eps1, eps2, eps3 without defining them.  The
reading used here (parity unpinned by the paper):

* Z~ = Z_near with every entry |z_ij| < eps1 |z_jj| of column j dropped;
* the pattern of column j of P is J_j = {i : |z_ij| >= eps2 |z_jj|};
* the rows taking part are I_j = the nonzero rows of Z~(:, J_j);
* p_j = argmin || e_j(I_j) - Z~(I_j, J_j) p ||_2   (plain least squares);
* entries |p_ij| < eps3 max_i |p_ij| are dropped afterwards.

Z_near is the Galerkin matrix restricted to the near field of the octree:
pairs of RWG functions whose leaf boxes (by edge midpoint) are at Chebyshev
distance <= 1.
"""
import numpy as np
import scipy.sparse as sp

from .rwg import build_rwg


def near_mask(V, F, nlv):
    """Boolean N x N mask of near pairs for a tree with nlv levels (level 0 =
    the bounding cube, enlarged by 1e-9, of the vertices)."""
    V = np.asarray(V, dtype=np.float64)
    r = build_rwg(V, F)
    mid = 0.5 * (V[r["edge"][:, 0]] + V[r["edge"][:, 1]])
    lo, hi = V.min(0), V.max(0)
    side = (hi - lo).max() * (1 + 1e-9)
    origin = 0.5 * (lo + hi) - 0.5 * side
    nside = 2 ** (nlv - 1)
    ijk = np.clip(np.floor((mid - origin) / (side / nside)).astype(int), 0, nside - 1)
    return np.abs(ijk[:, None, :] - ijk[None, :, :]).max(-1) <= 1


def sai(Zn, eps1, eps2, eps3):
    """Zn: dense N x N near-field matrix (zeros outside the near field).
    Returns P as a dense N x N array."""
    N = Zn.shape[0]
    d = np.abs(np.diag(Zn))
    Zt = np.where(np.abs(Zn) >= eps1 * d[None, :], Zn, 0.0)       # column-wise drop
    P = np.zeros_like(Zn)
    for j in range(N):
        col = Zn[:, j]
        J = np.flatnonzero((np.abs(col) >= eps2 * d[j]) & (col != 0))
        sub = Zt[:, J]
        I = np.flatnonzero(np.any(sub != 0, axis=1))
        A = sub[I, :]
        e = (I == j).astype(np.complex128)
        p, *_ = np.linalg.lstsq(A, e, rcond=None)
        keep = np.abs(p) >= eps3 * np.abs(p).max()
        P[J[keep], j] = p[keep]
    return P
