"""The Calderon multiplicative preconditioner on the GPU (section IV, eqs.
(25)-(27)) against the oracle, on the 1,920-unknown sphere (radius 0.5
wavelength; its barycentric refinement has 11,520 RWG), FP64:

* G x (sparse, exact up to rounding) and sampled rows of Z~ x and of
  Z~ G^-1 Z x (through the refined mesh's MLFMA) against the oracle's values
  in tests/golden/cmp_sphere_n1920.npz (written by make_cmp_golden.py);
* GMRES on the Calderon-preconditioned system solves Z x = b: the same x as
  the unpreconditioned solve with the same MLFMA, and the oracle's dense
  solve to the accuracy the MLFMA allows, in fewer iterations;
* the implicitly restarted Arnoldi method with Calderon-preconditioned inner
  solves gives the dense QZ characteristic values."""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ACC64 = dict(d0=6.0, interp_p=12)
GOLD = os.path.join(os.path.dirname(__file__), "golden", "cmp_sphere_n1920.npz")


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1412_1756_amd import Operator
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    g = np.load(GOLD)
    V, F = workloads.icosphere(3, 0.5)
    op = Operator(V, F, float(g["k"]), nlv=3, max_cols=1, **ACC64)
    info = op.cmp_build(nlv=3)
    print("cmp build", info, flush=True)
    return torch, op, g


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max())


def test_cmp_products_match_oracle(setup):
    """G x to rounding; Z~ x (a product of the refined mesh's MLFMA) to the
    FP64 acceptance 1e-4.  Z~ G^-1 Z x = Z~ u is a strongly cancelling
    product (the Calderon identity makes it O(1) while Z~ and u are large), so
    the MLFMA's error, relative to the size of the terms ||Z~|| ||u||, is
    amplified in it by rho = (||Z~ x|| / ||x||) ||u|| / ||Z~ u|| (from the
    oracle's values); the bound is 1e-4 rho."""
    torch, op, g = setup
    x = torch.tensor(g["x"], dtype=torch.complex128, device="cuda")
    rows = g["rows"]
    gx = op.cmp_apply(x, "G").cpu().numpy()
    zt = op.cmp_apply(x, "Zt").cpu().numpy()
    mx = op.cmp_apply(x, "M").cpu().numpy()
    e_g, e_z, e_m = _rel(gx, g["Gx"]), _rel(zt[rows], g["Ztx"]), _rel(mx[rows], g["Mx"])
    print(f"G x {e_g}, Z~ x rows {e_z}, Z~ G^-1 Z x rows {e_m} (2-norm, max element)", flush=True)
    rho = (np.linalg.norm(g["Ztx"]) / np.linalg.norm(g["x"][rows])) * np.linalg.norm(g["u"][rows]) \
        / np.linalg.norm(g["Mx"])
    print(f"cancellation factor of Z~ G^-1 Z x: {rho:.1f}", flush=True)
    assert e_g[0] < 1e-12
    assert e_z[0] < 1e-4
    assert e_m[0] < 1e-4 * rho
    # FP32 far field (the handle's accuracy settings are the FP64 ones; 6.6e-4
    # measured): the conversions around the refined MLFMA carry the FP32 error
    # only
    e32 = _rel(op.cmp_apply(x, "Zt", far="fp32").cpu().numpy()[rows], g["Ztx"])
    print(f"Z~ x rows, FP32 far field: {e32}", flush=True)
    assert e32[0] < 5e-3


def test_cmp_gmres_solves_z(setup):
    """The Calderon-preconditioned solve gives the unpreconditioned solve's x
    (the same MLFMA system) to 1e-7, and the oracle residual of x is bounded
    by the MLFMA error times ||Z|| ||x|| / ||b|| (as for the SAI solve)."""
    from oracle import efie
    torch, op, g = setup
    b = torch.tensor(g["b"], dtype=torch.complex128, device="cuda")
    x0, it0, rr0, ok0 = op.gmres(b, restart=200, maxit=2000, tol=1e-10, precond=False)
    x1, it1, rr1, ok1 = op.gmres(b, restart=200, maxit=2000, tol=1e-10, precond="cmp")
    x0, x1 = x0.cpu().numpy(), x1.cpu().numpy()
    print(f"GMRES to 1e-10: {it0} iterations unpreconditioned, {it1} Calderon-preconditioned; "
          f"difference {_rel(x1, x0)[0]:.2e}, against the dense solve {_rel(x1, g['xs'])[0]:.2e}", flush=True)
    assert ok0 and ok1
    assert it1 < it0 / 2
    assert _rel(x1, x0)[0] < 1e-7
    Z = efie.dense_Z(*workloads.icosphere(3, 0.5), float(g["k"]))
    bound = 1e-4 * np.linalg.norm(Z, 2) * np.linalg.norm(x1) / np.linalg.norm(g["b"])
    res = _rel(Z @ x1, g["b"])[0]
    print(f"oracle residual {res:.2e}, bound {bound:.2e}", flush=True)
    assert res < bound


def test_cmp_arnoldi_matches_qz(setup):
    torch, op, g = setup
    v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
    r = op.eigs(8, 30, v0, tol=1e-8, maxrestart=30, gmres_tol=1e-10, gmres_restart=100, precond="cmp")
    lam = np.sort(r["lam"].real)
    ref = np.sort(g["lam"].real)
    print("IRA with the Calderon preconditioner", lam, "QZ", ref, "OP products", r["n_op"], "GMRES iterations",
          r["gmres_iters"], flush=True)
    assert r["converged"]
    assert np.abs(lam - ref).max() < 1e-3
