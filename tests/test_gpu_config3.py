"""Finite differences in k of the GPU path with the tree and the angular
sampling frozen (k_sampling = k0, so that the handles differ only in their
k-dependent values: translators, phases, leaf patterns, near field):

* the operator: dZ/dk x of the dual pass on the 10 x 10 wavelength plate
  (29,800 unknowns, 6 levels, two-box buffer, FP64) against the central
  difference of Z x at k0 +- h and k0 +- 2h (h = 1e-4 k0), Richardson
  extrapolated;
* the characteristic values: d lambda/dk from cm_dlambda_dk on the
  1,920-unknown sphere (its TE1 and TE2 clusters, traced as cluster sums,
  which are smooth in k where single members of a degenerate cluster are
  not) against the same differences of the GPU's own Arnoldi eigenvalues."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K0 = 2 * np.pi
H = 1e-4 * K0


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _richardson(f):
    """d/dk at K0 from f(k): (4 D(h) - D(2h)) / 3 with the central
    differences D; returns (extrapolated, D(h))."""
    dh = (f(K0 + H) - f(K0 - H)) / (2 * H)
    d2h = (f(K0 + 2 * H) - f(K0 - 2 * H)) / (4 * H)
    return (4 * dh - d2h) / 3, dh


def test_config3_dzdk_matches_central_difference(torch_cuda):
    """The central difference with h = 1e-4 k carries a truncation error
    (h R)^2 / 6 of the phase exp(-i k R) over the plate's distances R up to
    14 wavelengths (about 1e-5, measured 2.3e-6 on the product); Richardson
    extrapolation over h and 2h removes it to O((h R)^4) ~ 1e-10, leaving the
    FP64 rounding of the products over 4h (about 1e-11 relative), so the
    extrapolated difference is bounded at 1e-7."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F, spec = workloads.workload("plate_10x10_n29800")
    acc = dict(nlv=6, d0=4.0, interp_p=10, wide_near=True, max_cols=2, k_sampling=K0)
    x = torch.tensor(workloads.cn01_block(29800, 2, 500), dtype=torch.complex128, device="cuda")
    op = Operator(V, F, K0, deriv=True, **acc)
    d = op.apply(x, "DZDK").cpu().numpy()
    del op

    def zx(k):
        return Operator(V, F, k, **acc).apply(x).cpu().numpy()

    fd, fd1 = _richardson(zx)
    e, e1 = relerr(d, fd), relerr(d, fd1)
    print(f"plate dZ/dk x vs central difference: h only {e1:.3e}, Richardson (h, 2h) {e:.3e}", flush=True)
    assert e < 1e-7


def test_dlambda_dk_matches_central_difference_of_gpu_eigenvalues(torch_cuda):
    """Cluster sums of d lambda/dk (TE1: 3 modes, TE2: 5) from the dZ/dk pass
    against the Richardson-extrapolated central difference of the cluster
    sums of the Arnoldi characteristic values at k0 +- h, k0 +- 2h (IRA
    tolerance 1e-9, inner GMRES 1e-10, so that the values carry about 1e-9
    of error and the difference about 1e-5 relative at most)."""
    torch = torch_cuda
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(3, 0.5)
    acc = dict(nlv=3, d0=6.0, interp_p=12, max_cols=8, k_sampling=K0)
    v0 = None

    def modes(k, deriv=False):
        nonlocal v0
        op = Operator(V, F, k, deriv=deriv, **acc)
        if v0 is None:
            v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
        op.sai_build()
        r = op.eigs(8, 30, v0, tol=1e-9, maxrestart=60, gmres_tol=1e-10, gmres_maxit=3000)
        print(f"k = {k:.10f}: nconv {r['nconv']}, restarts {r['restarts']}, inner failures {r['inner_failures']}, "
              f"largest Ritz residual {r['resid'].max():.1e}", flush=True)
        assert r["converged"], k
        o = np.argsort(r["lam"].real)
        return op, r["lam"].real[o], r["J"][:, o.tolist()]

    op, lam, J = modes(K0, deriv=True)
    te1, te2 = slice(0, 3), slice(3, 8)
    d1 = op.dlambda_dk(float(lam[te1].mean()), J[:, te1]).sum()
    d2 = op.dlambda_dk(float(lam[te2].mean()), J[:, te2]).sum()
    del op, J

    def sums(k):
        lm = modes(k)[1]
        return np.array([lm[te1].sum(), lm[te2].sum()])

    fd, fd1 = _richardson(sums)
    d = np.array([d1, d2])
    print(f"cluster sums of d lambda/dk {d}, central difference {fd1} (h), {fd} (Richardson)", flush=True)
    assert np.abs(d - fd).max() < 1e-4 * np.abs(fd).max()
