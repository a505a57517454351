"""Host logic of the mode tracker (paper_1412_1756_amd.tracking) on the CPU:
the library's products are replaced by dense oracle matrices of a small
plate, and the Arnoldi result by the oracle's QZ modes turned by arbitrary
complex phases and listed in a shuffled order.  The tracker must reproduce
the oracle's brute-force correspondence, characteristic values and
d lambda/dk."""
import numpy as np
import pytest
import torch

import workloads
from oracle import efie, modes

C0 = 299792458.0


class DenseOp:
    """Stand-in for Operator: apply() by dense oracle matrices on CPU tensors."""

    def __init__(self, V, F, k, seed):
        self.Z, self.dZ = efie.dense_Z(V, F, k, deriv=True)
        self.N = self.Z.shape[0]
        self.rng = np.random.default_rng(seed)

    def sai_build(self, *a):
        pass

    def apply(self, x, op="Z"):
        M = {"Z": self.Z, "R": self.Z.real, "X": self.Z.imag, "DZDK": self.dZ}[op]
        X = x.numpy().reshape(self.N, -1)
        y = torch.tensor(M @ X, dtype=torch.complex128)
        return y.reshape(-1) if x.dim() == 1 else y

    def eigs(self, nev, ncv, v0, **kw):
        lam, J = modes.qz_modes(self.Z.imag, self.Z.real, nev=nev, vectors=True)
        sh = self.rng.permutation(nev)
        ph = np.exp(1j * self.rng.uniform(0, 2 * np.pi, nev)) * self.rng.uniform(0.5, 2.0, nev)
        Jc = (J * ph[None, :])[:, sh]
        return dict(lam=lam[sh], J=torch.tensor(Jc), converged=True, n_op=0, inner_retries=0)

    def jd(self, nev, v0, **kw):
        r = self.eigs(nev, 0, v0)
        return dict(lam=r["lam"].real, J=r["J"], nconv=nev, converged=True, n_matvec=0)

    # the library's mode post-processing, written out densely from its
    # definitions (cm_real_currents, cm_modal_correlation, cm_dlambda_dk)
    def real_currents(self, J):
        Jn = J.numpy()
        ph = np.exp(-0.5j * np.angle((Jn * Jn).sum(0)))
        Jr = (Jn * ph[None, :]).real
        RJ = self.Z.real @ Jr
        nrm = np.sqrt((Jr * RJ).sum(0))
        return (torch.tensor(Jr / nrm[None, :], dtype=torch.complex128),
                torch.tensor(RJ / nrm[None, :], dtype=torch.complex128))

    def modal_correlation(self, Ja, Jb):
        A, B = Ja.numpy(), Jb.numpy()
        R = self.Z.real
        na = np.abs(np.einsum("ia,ia->a", A, R @ A))
        nb = np.abs(np.einsum("ib,ib->b", B, R @ B))
        return np.abs(A.T @ (R @ B)) / np.sqrt(na[:, None] * nb[None, :])

    def dlambda_dk(self, lam, J):
        j = J.numpy().real.reshape(self.N, -1)
        return np.atleast_1d(modes.dlambda_dk(j, np.atleast_1d(lam), self.dZ.imag, self.dZ.real, self.Z.real))


@pytest.mark.parametrize("solver", ["ira", "jd"])
def test_tracker_matches_oracle_on_dense_plate(solver):
    from paper_1412_1756_amd.tracking import track_modes
    V, F = workloads.plate(10, 6, 0.1)
    ks = [2 * np.pi * f / C0 for f in (280e6, 300e6, 320e6)]
    nev, ntrack = 6, 4
    ops = {}

    def make_op(k):
        ops[k] = DenseOp(V, F, k, seed=len(ops))
        return ops[k]

    t = track_modes(make_op, ks, nev, 20, None, ntrack=ntrack, solver=solver)
    # oracle correspondence, independent of the tracker
    Jp, lam_o, d_o = None, [], []
    for k in ks:
        Z, dZ = ops[k].Z, ops[k].dZ
        lo, Jo = modes.qz_modes(Z.imag, Z.real, nev=nev, vectors=True)
        lo = lo.real
        p = np.arange(ntrack) if Jp is None else modes.track_by_correlation(Jp, Jo, Z.real)[0]
        lam_o.append(lo[p])
        d_o.append(modes.dlambda_dk(Jo[:, p], lo[p], dZ.imag, dZ.real, Z.real))
        Jp = Jo[:, p]
    np.testing.assert_allclose(t["lam"], np.array(lam_o), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(t["dldk"], np.array(d_o), rtol=1e-6)
    assert t["corr"].min() > 0.9
    # first-order predictions land within a fraction of each step
    step = np.abs(t["lam"][1:] - t["lam"][:-1])
    assert np.all(np.abs(t["lam"][1:] - t["pred"]) < 0.5 * step + 1e-9)
