"""Characteristic modes followed over a wavenumber sweep (the plate sweep of
section V, where each characteristic value is plotted against frequency).

At every wavenumber: the SAI build, the implicitly restarted Arnoldi solve
(cm_eigs), real R-normalised currents and d lambda/dk per mode from the dZ/dk
pass.  Between consecutive wavenumbers the modes are matched by modal
correlation |J_a(k_i)^T R(k_{i+1}) J_b(k_{i+1})| of R-normalised real
currents, maximised over all one-to-one correspondences (a linear assignment
of an nev x nev matrix).  Every product with Z, R and dZ/dk runs in the
library; the host handles the nev x nev matrices and N x nev dot products.
Modes are assumed non-degenerate (inside a degenerate cluster the
correspondence is arbitrary).
"""
import numpy as np
import torch
from scipy.optimize import linear_sum_assignment

from .autograd import dlambda_dk


def real_currents(op, J):
    """Real currents J^T R J = 1 from IRA eigenvectors (N x m complex128 CUDA
    tensor; each column a real vector times a complex scalar): the column is
    turned by the phase that makes sum_i J_i^2 real and positive, its real
    part kept and scaled.  Returns (J, R J) as N x m complex128 CUDA tensors
    with zero imaginary parts."""
    ph = torch.exp(-0.5j * torch.angle((J * J).sum(0)))
    Jr = (J * ph[None, :]).real.to(torch.complex128).contiguous()
    RJ = op.apply(Jr, "R")
    nrm = torch.sqrt((Jr.real * RJ.real).sum(0))
    return Jr / nrm[None, :], RJ / nrm[None, :]


def track_modes(make_op, ks, nev, ncv, v0, ntrack=None, sai=(0.01, 0.014, 0.18), solver="ira", **eig_kw):
    """Follow the ntrack (<= nev, default nev) smallest-|lambda| modes of
    ks[0] through the sweep ks; each eigen-solve computes nev modes, the
    spare ones being candidates for a mode whose |lambda| rank changes.
    solver: "ira" (Operator.eigs on Z^-1 R, ncv Arnoldi vectors) or "jd"
    (Operator.jd on the pencil (X, R) with target 0; ncv is unused, eig_kw
    goes to Operator.jd).

    make_op(k) returns an Operator at wavenumber k built with deriv=True and
    max_cols >= nev (the caller chooses mesh, levels and accuracy); v0 is the
    complex128 CUDA start vector of every Arnoldi solve; eig_kw goes to
    Operator.eigs.  Returns a dict:
      lam   [n_k, ntrack]      characteristic value of track a at ks[i]
      dldk  [n_k, ntrack]      its d lambda/dk
      corr  [n_k - 1, ntrack]  modal correlation of each step's match
      pred  [n_k - 1, ntrack]  lam[i] + dldk[i] (ks[i+1] - ks[i]), the
                               first-order prediction the match can be
                               checked against
      index [n_k, ntrack]      column of the Arnoldi result (sorted by
                               |lambda|) each track took
      converged, n_op, inner_retries
                               per wavenumber (Operator.eigs; for "jd" n_op
                               counts operator applies)
    """
    ks = [float(k) for k in ks]
    n = len(ks)
    m = nev if ntrack is None else int(ntrack)
    if not 1 <= m <= nev:
        raise ValueError("ntrack must be in 1..nev")
    lam_t = np.zeros((n, m))
    d_t = np.zeros((n, m))
    idx_t = np.zeros((n, m), dtype=np.int64)
    corr = np.zeros((max(n - 1, 0), m))
    pred = np.zeros((max(n - 1, 0), m))
    conv, nops, retries = [], [], []
    Jprev = None
    for i, k in enumerate(ks):
        op = make_op(k)
        op.sai_build(*sai)
        if solver == "ira":
            r = op.eigs(nev, ncv, v0, **eig_kw)
            nops.append(int(r["n_op"]))
            retries.append(int(r["inner_retries"]))
        elif solver == "jd":
            r = op.jd(nev, v0, **eig_kw)
            nops.append(int(r["n_matvec"]))
            retries.append(0)
            if r["nconv"] < nev:
                raise RuntimeError(f"Jacobi-Davidson found {r['nconv']} of {nev} modes at k = {k}")
        else:
            raise ValueError("solver must be 'ira' or 'jd'")
        conv.append(bool(r["converged"]))
        lam = np.real(r["lam"])
        order = np.argsort(np.abs(lam))
        lam = lam[order]
        J, RJ = real_currents(op, r["J"][:, order.tolist()])
        d = np.array([dlambda_dk(op, lam[j], J[:, j])[0] for j in range(nev)])
        if Jprev is None:
            perm = np.arange(m)
        else:
            # correlations with R at this wavenumber; the new currents are
            # R-normalised here, the previous ones are normalised by R J_prev
            RJp = op.apply(Jprev, "R").real.cpu().numpy()
            Jp = Jprev.real.cpu().numpy()
            C = np.abs(Jp.T @ RJ.real.cpu().numpy()) / np.sqrt(np.sum(Jp * RJp, axis=0))[:, None]
            rows, cols = linear_sum_assignment(-C)          # m x nev, m <= nev
            perm = cols[np.argsort(rows)]
            corr[i - 1] = C[np.arange(m), perm]
            pred[i - 1] = lam_t[i - 1] + d_t[i - 1] * (k - ks[i - 1])
        lam_t[i] = lam[perm]
        d_t[i] = d[perm]
        idx_t[i] = perm
        Jprev = J[:, perm.tolist()].contiguous()
        del op, r, RJ
    return dict(k=np.array(ks), lam=lam_t, dldk=d_t, corr=corr, pred=pred, index=idx_t, converged=conv,
                n_op=nops, inner_retries=retries)
