"""GPU tests of the library's mode post-processing and preconditioner entry
points against the oracle's dense matrices on the 1,920-unknown sphere:
cm_vdot, cm_real_currents, cm_modal_correlation, cm_dlambda_dk, the SAI of
X_near with the preconditioned X^-1 R route, and per-wavenumber SAIs of a
sweep handle.  Argument errors of these calls come back as status codes."""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K0 = 2 * np.pi
ACC64 = dict(d0=6.0, interp_p=12)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def cfg1():
    from oracle import efie
    V, F = workloads.icosphere(3, 0.5)
    Z, dZ = efie.dense_Z(V, F, K0, deriv=True)
    return V, F, Z, dZ


def _op(V, F, **kw):
    from paper_1412_1756_amd import Operator
    return Operator(V, F, kw.pop("k", K0), nlv=3, **ACC64, **kw)


def test_vdot_matches_numpy(torch_cuda, cfg1):
    torch = torch_cuda
    V, F, Z, _ = cfg1
    op = _op(V, F, max_cols=4)
    x = workloads.cn01_block(op.N, 3, 40)
    y = workloads.cn01_block(op.N, 3, 50)
    ref = np.vdot(x, y)
    for dt, tol in ((torch.complex128, 1e-13), (torch.complex64, 1e-6)):
        X = torch.tensor(x, dtype=dt, device="cuda")
        Y = torch.tensor(y, dtype=dt, device="cuda")
        v = complex(op.vdot(X, Y).cpu())
        print(f"vdot {dt}: {abs(v - ref) / abs(ref):.2e}", flush=True)
        assert abs(v - ref) < tol * np.linalg.norm(x) * np.linalg.norm(y)
        # a column slice of a wider tensor (row stride 3, 2 columns)
        v2 = complex(op.vdot(X[:, 1:], Y[:, 1:]).cpu())
        r2 = np.vdot(x[:, 1:], y[:, 1:])
        assert abs(v2 - r2) < tol * np.linalg.norm(x) * np.linalg.norm(y)


def test_real_currents_and_modal_correlation(torch_cuda, cfg1):
    """Real R-normalised currents from phase-rotated QZ eigenvectors, and the
    correlation matrix, against the same definitions on the dense oracle R."""
    torch = torch_cuda
    from oracle import modes
    V, F, Z, _ = cfg1
    R = Z.real
    op = _op(V, F, max_cols=4)
    lam, J = modes.qz_modes(Z.imag, R, nev=6, vectors=True)
    rng = np.random.default_rng(7)
    Jc = J * (np.exp(1j * rng.uniform(0, 2 * np.pi, 6)) * rng.uniform(0.5, 2.0, 6))[None, :]
    Jr, RJ = op.real_currents(torch.tensor(Jc, dtype=torch.complex128, device="cuda"))
    Jr, RJ = Jr.cpu().numpy(), RJ.cpu().numpy()
    assert np.abs(Jr.imag).max() == 0.0
    # reference: the same phase rule and normalisation with the dense R
    ph = np.exp(-0.5j * np.angle((Jc * Jc).sum(0)))
    Jo = (Jc * ph[None, :]).real
    Jo /= np.sqrt(np.einsum("ia,ij,ja->a", Jo, R, Jo))[None, :]
    e = relerr(Jr.real, Jo)
    print(f"real currents {e:.2e}; J^T R J diag", np.diag(Jr.real.T @ R @ Jr.real), flush=True)
    assert e < 1e-7
    assert relerr(RJ.real, R @ Jr.real) < 1e-7
    Cg = op.modal_correlation(torch.tensor(Jr, device="cuda"), torch.tensor(Jc, dtype=torch.complex128,
                                                                               device="cuda"))
    Co = np.abs(Jr.real.T @ R @ Jc) / np.sqrt(np.abs(np.einsum("ia,ij,ja->a", Jr.real, R, Jr.real))[:, None]
                                              * np.abs(np.einsum("ib,ij,jb->b", Jc, R, Jc))[None, :])
    print("correlation max err", np.abs(Cg - Co).max(), flush=True)
    assert np.abs(Cg - Co).max() < 1e-7
    # currents of different characteristic values are R-orthogonal (the
    # first three are the TE1 cluster, the rest of TE2; inside a degenerate
    # cluster QZ returns no particular basis): the correlation of the set
    # with itself is 1 on the diagonal and 0 between the clusters
    Cs = op.modal_correlation(torch.tensor(Jr, device="cuda"), torch.tensor(Jr, device="cuda"))
    assert np.abs(np.diag(Cs) - 1).max() < 1e-12
    assert np.abs(Cs[:3, 3:]).max() < 1e-6


def test_dlambda_dk_single_mode_against_oracle(torch_cuda, cfg1):
    """cm_dlambda_dk for single QZ modes (m = 1) and for a cluster (m = 3),
    against the oracle's formula on the dense dZ/dk."""
    torch = torch_cuda
    from oracle import modes
    V, F, Z, dZ = cfg1
    op = _op(V, F, max_cols=4, deriv=True)
    lam, J = modes.qz_modes(Z.imag, Z.real, nev=8, vectors=True)
    lam = lam.real
    o = np.argsort(lam)
    lam, J = lam[o], J[:, o]
    for j in (3, 5):
        d = op.dlambda_dk(lam[j], torch.tensor(J[:, j] * np.exp(0.3j), dtype=torch.complex128, device="cuda"))
        do = modes.dlambda_dk(J[:, [j]].real, lam[[j]], dZ.imag, dZ.real, Z.real)
        print(f"mode {j}: {d[0]:.8f} oracle {do[0]:.8f}", flush=True)
        assert abs(d[0] - do[0]) < 1e-6 * max(1.0, abs(do[0]))
    d3 = op.dlambda_dk(float(np.mean(lam[:3])), torch.tensor(J[:, :3], dtype=torch.complex128, device="cuda"))
    do3 = modes.dlambda_dk_cluster(J[:, :3].real, lam[:3], dZ.imag, dZ.real, Z.real)
    print("cluster", d3, do3, flush=True)
    assert np.abs(d3 - do3).max() < 1e-6 * np.abs(do3).max()


def test_sai_of_x_matches_oracle_and_preconditions_x_solves(torch_cuda, cfg1):
    """The SAI of X_near (part X): entries against the oracle's least squares
    on Im of its own near field, and the preconditioned X^-1 R Arnoldi route
    against dense QZ with fewer inner GMRES iterations than unpreconditioned."""
    torch = torch_cuda
    from oracle import modes
    from oracle.sai import near_mask, sai
    V, F, Z, _ = cfg1
    op = _op(V, F, max_cols=1)
    eps = (0.01, 0.014, 0.18)
    op.sai_build(*eps, part="X")
    Pg = op.export_near(3).toarray()
    Po = sai(np.where(near_mask(V, F, 3), Z.imag, 0).astype(np.complex128), *eps)
    both = (Pg != 0) & (Po != 0)
    assert both.sum() >= 0.999 * max(np.count_nonzero(Pg), np.count_nonzero(Po))
    assert np.abs(Pg[both] - Po[both]).max() < 1e-9 * np.abs(Po).max()
    assert np.abs(Pg.imag).max() == 0.0
    x = workloads.cn01(op.N, 0)
    y = op.sai_apply(torch.tensor(x, dtype=torch.complex128, device="cuda"), part="X").cpu().numpy()
    assert relerr(y, Pg @ x) < 1e-12
    v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
    kw = dict(tol=1e-8, maxrestart=30, gmres_tol=1e-10, gmres_maxit=2000, route="X", vectors=False)
    rp = op.eigs(8, 30, v0, precond=True, **kw)
    ru = op.eigs(8, 30, v0, precond=False, **kw)
    lo = np.sort(modes.qz_modes(Z.imag, Z.real, nev=8).real)
    print("X^-1 R with SAI(X):", np.sort(rp["lam"].real), "GMRES", rp["gmres_iters"], "without:", ru["gmres_iters"],
          flush=True)
    assert rp["converged"] and rp["inner_failures"] == 0
    assert np.abs(np.sort(rp["lam"].real) - lo).max() < 1e-3
    assert rp["gmres_iters"] < ru["gmres_iters"]


def test_sai_per_wavenumber_on_a_sweep_handle(torch_cuda, cfg1):
    """A two-wavenumber handle keeps one SAI per wavenumber: built at k[1], its
    apply (k_index 1) equals a single-wavenumber handle's at that k bit for
    bit; columns at k[0] without an SAI there are refused."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator, _lib
    from paper_1412_1756_amd._lib import CmError
    V, F, Z, _ = cfg1
    k1 = 1.05 * K0
    sw = Operator(V, F, [K0, k1], nlv=3, **ACC64, max_cols=8)
    one = _op(V, F, k=k1, max_cols=8)
    sw.sai_build(k_index=1)
    one.sai_build()
    X = torch.tensor(workloads.cn01_block(sw.N, 2, 60), dtype=torch.complex128, device="cuda")
    ys = sw.sai_apply(X, k_index=[1, 1])
    yo = one.sai_apply(X)
    assert torch.equal(ys, yo)
    with pytest.raises(CmError) as e:
        sw.sai_apply(X, k_index=[0, 1])
    assert e.value.code == _lib.CM_E_NOT_BUILT
    # mixed wavenumbers: each column through its wavenumber's P (the gathered
    # batch has another width, so the row sums may be grouped differently)
    sw.sai_build(k_index=0)
    zero = _op(V, F, max_cols=8)
    zero.sai_build()
    ym = sw.sai_apply(X, k_index=[0, 1]).cpu().numpy()
    assert relerr(ym[:, 1], yo[:, 1].cpu().numpy()) < 1e-14
    assert relerr(ym[:, 0], zero.sai_apply(X).cpu().numpy()[:, 0]) < 1e-14


def test_mode_call_argument_errors(torch_cuda, cfg1):
    torch = torch_cuda
    from paper_1412_1756_amd import _lib
    L = _lib.lib()
    V, F, Z, _ = cfg1
    op = _op(V, F, max_cols=2)
    N = op.N
    J = torch.zeros((N, 2), dtype=torch.complex128, device="cuda")
    Jo = torch.zeros_like(J)
    RJ = torch.zeros_like(J)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    jp, op_, rp = C.c_void_p(J.data_ptr()), C.c_void_p(Jo.data_ptr()), C.c_void_p(RJ.data_ptr())
    d = np.zeros(2)
    Cm = np.zeros(4)
    assert L.cm_dlambda_dk(op._h, 0.1, jp, 2, 2, d.ctypes.data, s) == _lib.CM_E_NOT_BUILT   # no CM_FLAG_DERIV
    assert L.cm_real_currents(op._h, jp, 2, 0, op_, rp, 2, s) == _lib.CM_E_BADARG         # m = 0
    assert L.cm_real_currents(op._h, jp, 1, 2, op_, rp, 2, s) == _lib.CM_E_BADARG         # ldj < m
    assert L.cm_real_currents(op._h, jp, 2, 2, jp, rp, 2, s) == _lib.CM_E_BADARG         # aliasing
    assert L.cm_real_currents(op._h, jp, 2, 2, op_, rp, 2, s) == _lib.CM_E_NUMERIC        # zero currents
    assert L.cm_modal_correlation(op._h, jp, 2, 2, jp, 1, 2, Cm.ctypes.data, s) == _lib.CM_E_BADARG
    assert L.cm_sai_build(op._h, 0.01, 0.014, 0.18, 1, 1.0) == _lib.CM_E_BADARG           # k_index >= n_k
    assert L.cm_sai_build(op._h, 0.01, 0.014, 0.18, 0, -0.5) == _lib.CM_E_BADARG          # tau < 0
    assert L.cm_sai_apply(op._h, jp, rp, 2, 2, None, 1.0, 1, s) == _lib.CM_E_NOT_BUILT    # no SAI yet
    out = torch.zeros((), dtype=torch.complex128, device="cuda")
    assert L.cm_vdot(op._h, jp, rp, 1, 2, 1, C.c_void_p(out.data_ptr()), s) == _lib.CM_E_BADARG   # ld < ncols
    # the Python layer checks out / v0 before any call
    x = torch.zeros(N, dtype=torch.complex128, device="cuda")
    with pytest.raises(TypeError):
        op.apply(x, out=torch.zeros(N, dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError):
        op.apply(x, out=torch.zeros(N - 1, dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        op.eigs(2, 6, torch.zeros(N - 1, dtype=torch.complex128, device="cuda"), precond=False)
    with pytest.raises(TypeError):
        op.eigs(2, 6, torch.zeros(N, dtype=torch.complex64, device="cuda"), precond=False)
