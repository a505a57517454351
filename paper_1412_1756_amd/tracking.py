"""Characteristic modes followed over a wavenumber sweep (the plate sweep of
section V, where each characteristic value is plotted against frequency).

At every wavenumber: the SAI build, the eigen-solve (IRA, cm_eigs, or
Jacobi-Davidson, cm_jd), real R-normalised currents (cm_real_currents) and
d lambda/dk per mode from the dZ/dk pass (cm_dlambda_dk).  Between
consecutive wavenumbers the modes are matched by modal correlation
|J_a(k_i)^T R(k_{i+1}) J_b(k_{i+1})| of R-normalised real currents
(cm_modal_correlation), maximised over all one-to-one correspondences (a
linear assignment of an nev x nev matrix on the host).  Every product and
every N-vector reduction runs in the library; the host handles only the
nev x nev matrices.  Modes are assumed non-degenerate (inside a degenerate
cluster the correspondence is arbitrary).
"""
import numpy as np
from scipy.optimize import linear_sum_assignment


def real_currents(op, J):
    """Real currents J^T R J = 1 from eigenvectors (N x m complex128 CUDA
    tensor; each column a real vector times a complex scalar): the column is
    turned by the phase that makes sum_i J_i^2 real and positive, its real
    part kept and scaled (cm_real_currents).  Returns (J, R J) as N x m
    complex128 CUDA tensors with zero imaginary parts."""
    return op.real_currents(J)


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
        d = np.array([op.dlambda_dk(lam[j], J[:, j])[0] for j in range(nev)])
        if Jprev is None:
            perm = np.arange(m)
        else:
            # correlations with R at this wavenumber (both sets normalised by
            # their R-norms at this wavenumber)
            C = op.modal_correlation(Jprev, J)
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
