"""Characteristic modes of the 1,966,080-unknown sphere (radius 12
wavelengths, 8 levels, FP32 far field with the FP64 near field, FP64
Arnoldi): the implicitly restarted Arnoldi method on Z^-1 R (eq. (24)) for 20
modes with inner GMRES solves (tolerance 1e-3, the paper's), bounded by the
size of the factorisation (CM_CONFIG5_NCV, default 60, the paper's order),
the number of restarts (CM_CONFIG5_RESTARTS, default 3) and the inner
iterations per solve (CM_CONFIG5_GMRES_MAXIT, default 400).  The inner
solves are unpreconditioned unless CM_CONFIG5_PRECOND=sai: at this size the
SAI of Z_near (the thresholds' reading of the build) slows GMRES down (300
preconditioned iterations leave the residual above 1e-3 where about 265
unpreconditioned ones reach it).

ka = 24 pi lies 1e-4 (relative) from the TM_26 interior resonance of the
EFIE, so Z is nearly singular there and the inner solves may stop at their
iteration bound; the run then measures how far the method gets rather than
asserting convergence.  No dense solver reaches this size, so the eight Ritz
pairs of smallest Ritz residual are checked by

* parity of the products the residuals are computed from: rows S of
  Z J = R J + i X J from the FP64 applies against the same rows of the
  oracle's Z (filled by CPU worker processes while the GPU solves), relative
  to their norm (X J alone is small where lambda is, so its own relative
  error is larger);
* the pencil residual ||X J - lambda R J|| / (||X J|| + |lambda| ||R J||)
  of every pair from the FP64 applies, reported, and the closed-form
  characteristic values of the sphere as a band for the pairs whose residual
  is below 1e-3 (the faceted mesh shifts them by about |d lambda/d(ka)| times
  the change of the effective ka).

The run takes minutes of GPU time, so it runs only with CM_CONFIG5_EIGS=1;
its printed summary (also written as JSON to $CM_CONFIG5_OUT when set) is what
the performance record quotes."""
import json
import multiprocessing as mp
import os
import time

import numpy as np
import pytest

import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("CM_CONFIG5_EIGS") != "1",
                                 reason="tens of minutes of GPU time: set CM_CONFIG5_EIGS=1 to run")]

K0 = 2 * np.pi
NEV = 20
NCV = int(os.environ.get("CM_CONFIG5_NCV", "60"))
NROWS = 8


def _oracle_rows(args):
    name, row, out = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import efie
    V, F, spec = workloads.workload(name)
    Zr = efie.rows_Z(V, F, spec["k"], np.array([row]))
    np.save(out, Zr[0])
    return row


def test_config5_twenty_modes():
    import torch
    from oracle import modes
    from paper_1412_1756_amd import Operator
    assert torch.cuda.is_available()
    name = "sphere_r12_n1966080"
    V, F, spec = workloads.workload(name)
    N = 1966080
    rows = np.sort(np.random.default_rng(2).choice(N, NROWS, replace=False))
    tmp = os.environ.get("TMPDIR", "/tmp")
    paths = [os.path.join(tmp, f"cm_cfg5_row_{r}.npy") for r in rows]
    t0 = time.time()
    op = Operator(V, F, K0, nlv=8, d0=4.5, interp_p=10, max_cols=8, verbose=True)
    t_create = time.time() - t0
    t0 = time.time()
    precond = os.environ.get("CM_CONFIG5_PRECOND", "none") == "sai"
    if precond:
        op.sai_build(0.01, 0.014, 0.18)
    t_sai = time.time() - t0
    print(f"cfg5: create {t_create:.1f} s, SAI of Z_near {t_sai:.1f} s ({op.sai_nnz() if precond else 0} entries)",
          flush=True)
    # the oracle rows are filled on the host while the GPU solves
    pool = mp.get_context("spawn").Pool(NROWS)
    pending = pool.map_async(_oracle_rows, [(name, int(r), p) for r, p in zip(rows, paths)])
    v0 = torch.tensor(workloads.cn01(N, 3), dtype=torch.complex128, device="cuda")
    t0 = time.time()
    r = op.eigs(NEV, NCV, v0, tol=1e-6, maxrestart=int(os.environ.get("CM_CONFIG5_RESTARTS", "3")),
                gmres_restart=200, gmres_maxit=int(os.environ.get("CM_CONFIG5_GMRES_MAXIT", "400")),
                gmres_tol=float(os.environ.get("CM_CONFIG5_GMRES_TOL", "1e-3")), far="fp32", precond=precond)
    t_eigs = time.time() - t0
    lam = r["lam"]
    o = np.argsort(np.abs(lam))
    lam, resid = lam[o], r["resid"][o]
    nconv = int(r["nconv"])
    print(f"cfg5: IRA {t_eigs:.1f} s, {nconv} of {NEV} converged, {r['n_op']} OP products, {r['gmres_iters']} GMRES "
          f"iterations ({r['gmres_iters'] / max(1, r['n_op']):.1f} per Arnoldi step, {r['inner_failures']} solves "
          f"missed the tolerance), {r['restarts']} restarts", flush=True)
    print("lambda", np.round(lam.real, 7), flush=True)
    best = np.argsort(resid)[:8]            # the checks cover the eight best Ritz pairs
    J = r["J"][:, o.tolist()][:, best.tolist()]
    lc = lam.real[best]
    Jr, RJ = op.real_currents(J)
    XJ = op.apply(Jr, "X")
    pres_gpu = np.array([(torch.linalg.vector_norm(XJ[:, j] - lc[j] * RJ[:, j])
                          / (torch.linalg.vector_norm(XJ[:, j]) + abs(lc[j]) * torch.linalg.vector_norm(RJ[:, j]))).item()
                         for j in range(best.size)])
    Jh = Jr.real.cpu().numpy()
    XS = XJ[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    RS = RJ[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    del J, Jr, RJ, XJ, op
    pending.get(timeout=3600)
    pool.close()
    Zr = np.stack([np.load(p) for p in paths])
    for p in paths:
        os.remove(p)
    Xo, Ro = Zr.imag @ Jh, Zr.real @ Jh
    ex = np.linalg.norm(XS - Xo) / np.linalg.norm(Xo)
    er = np.linalg.norm(RS - Ro) / np.linalg.norm(Ro)
    ez = np.linalg.norm((RS + 1j * XS) - (Ro + 1j * Xo)) / np.linalg.norm(Ro + 1j * Xo)
    pres_rows = np.linalg.norm(Xo - lc[None, :] * Ro, axis=0) / (np.linalg.norm(Xo, axis=0)
                                                                 + np.abs(lc) * np.linalg.norm(Ro, axis=0))
    cf = modes.sphere_spectrum(K0 * 12.0, nmax=120)
    near = [min(cf, key=lambda t: abs(t[0] - l)) for l in lc]
    summary = dict(workload=name, N=N, nev=NEV, ncv=NCV, nconv=nconv, t_create_s=t_create, t_sai_s=t_sai,
                   t_eigs_s=t_eigs, n_op=r["n_op"], gmres_iters=r["gmres_iters"], restarts=r["restarts"],
                   inner_failures=r["inner_failures"],
                   gmres_per_arnoldi_step=r["gmres_iters"] / max(1, r["n_op"]),
                   eigenmodes_per_hour=3600.0 * nconv / (t_create + t_sai + t_eigs),
                   lam_all=lam.real.tolist(), ritz_resid=resid.tolist(), checked=best.tolist(),
                   lam=lc.tolist(), pencil_residual=pres_gpu.tolist(), pencil_residual_rows=pres_rows.tolist(),
                   rows_err_X=ex, rows_err_R=er, rows_err_Z=ez, precond="sai" if precond else "none",
                   closed_form=[(float(t[0]), t[1], t[2]) for t in near], rows=rows.tolist())
    print(json.dumps(summary), flush=True)
    if os.environ.get("CM_CONFIG5_OUT"):
        with open(os.environ["CM_CONFIG5_OUT"], "w") as f:
            json.dump(summary, f, indent=1)
        np.savez(os.environ["CM_CONFIG5_OUT"] + ".npz", XS=XS, RS=RS, Xo=Xo, Ro=Ro, lam=lc)
    # the FP64 applies behind the residuals agree with the oracle's rows (the
    # FP64 far field at these settings: a few 1e-4)
    assert ez < 1e-3 and er < 1e-3, (ez, er)
    # pairs that did converge in the pencil sense lie in the closed-form band
    ok = pres_gpu < 1e-3
    assert all(abs(t[0] - l) < 2e-3 for t, l, g in zip(near, lc, ok) if g)
