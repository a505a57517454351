"""Characteristic values: dense QZ of the pencil (X, R) (eq. (6)) and the
closed-form values of the PEC sphere.

Closed forms (Harrington-Mautz characteristic values of a PEC sphere of radius
a, x = ka, modal degeneracy 2n + 1):

  TE_n:  lambda = -y_n(x) / j_n(x)
  TM_n:  lambda = -[x y_n(x)]' / [x j_n(x)]'

with j_n, y_n the spherical Bessel and Neumann functions.  Their
k-derivatives follow from the Wronskian j_n y_n' - j_n' y_n = 1/x^2:

  d lambda_TE / dk = -a / (x^2 j_n(x)^2)
  d lambda_TM / dk = a (n(n+1)/x^2 - 1) / ([x j_n(x)]')^2

Table II of the paper lists values with this sign convention (negative for the
electric-energy modes).

Mode tracking over a frequency sweep (the plate sweep of section V follows
each characteristic value from one frequency to the next; the paper does not
say how modes are matched): modal correlation of the R-normalised real
currents, maximised over all correspondences.
"""
import numpy as np
import scipy.linalg as sl
from scipy.special import spherical_jn, spherical_yn


def qz_modes(X, R, nev=None, vectors=False):
    """Finite characteristic values sorted by |lambda| (and R-normalised real
    eigenvectors when vectors=True)."""
    if vectors:
        a_b, J = sl.eig(X, R, right=True, homogeneous_eigvals=True)
    else:
        a_b = sl.eig(X, R, right=False, homogeneous_eigvals=True)
    a, b = a_b
    scale = np.abs(a).max()
    fin = np.abs(b) > 1e-10 * scale
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = a[fin] / b[fin]
    order = np.argsort(np.abs(lam))
    lam = lam[order]
    if nev is not None:
        lam = lam[:nev]
    if not vectors:
        return lam
    J = J[:, fin][:, order]
    if nev is not None:
        J = J[:, :nev]
    J = np.real(J * np.exp(-1j * np.angle(J[np.argmax(np.abs(J), axis=0), np.arange(J.shape[1])])))
    J /= np.sqrt(np.einsum("in,ij,jn->n", J, R, J))[None, :]
    return lam, J


def sphere_cv(n: int, x: float, kind: str) -> float:
    if kind == "TE":
        return -spherical_yn(n, x) / spherical_jn(n, x)
    djx = spherical_jn(n, x) + x * spherical_jn(n, x, derivative=True)
    dyx = spherical_yn(n, x) + x * spherical_yn(n, x, derivative=True)
    return -dyx / djx


def sphere_dcv_dk(n: int, k: float, a: float, kind: str) -> float:
    x = k * a
    if kind == "TE":
        return -a / (x * x * spherical_jn(n, x) ** 2)
    djx = spherical_jn(n, x) + x * spherical_jn(n, x, derivative=True)
    return a * (n * (n + 1) / (x * x) - 1.0) / djx ** 2


def sphere_spectrum(x: float, nmax: int = 40):
    """All closed-form (lambda, kind, n, degeneracy) sorted by |lambda|."""
    out = []
    for n in range(1, nmax + 1):
        for kind in ("TE", "TM"):
            out.append((sphere_cv(n, x, kind), kind, n, 2 * n + 1))
    out.sort(key=lambda t: abs(t[0]))
    return out


def sphere_smallest(x: float, count: int, nmax: int = 40):
    """The `count` smallest-|lambda| closed-form values with multiplicity."""
    vals = []
    for lam, kind, n, deg in sphere_spectrum(x, nmax):
        vals.extend([lam] * deg)
        if len(vals) >= count:
            break
    return np.array(vals[:count])


def dlambda_dk(J, lam, dX, dR, R):
    """d lambda/dk = J^T (dX - lambda dR) J / J^T R J for real J (one mode
    per column)."""
    num = np.einsum("in,ij,jn->n", J, dX, J) - lam * np.einsum("in,ij,jn->n", J, dR, J)
    return num / np.einsum("in,ij,jn->n", J, R, J)


def dlambda_dk_cluster(J, lam, dX, dR, R):
    """Derivatives of a degenerate cluster: eigenvalues of the projected
    matrix Ja^T (dX - lambda dR) Jb with R-orthonormalised J."""
    Rc = J.T @ R @ J
    Lc = np.linalg.cholesky(Rc)
    Q = J @ np.linalg.inv(Lc).T
    M = Q.T @ (dX - np.mean(lam) * dR) @ Q
    return np.sort(np.linalg.eigvalsh(0.5 * (M + M.T)))


def modal_correlation(Ja, Jb, R):
    """|Ja^T R Jb| normalised by the R-norms of the columns: 1 for the same
    real current, 0 for R-orthogonal ones (characteristic currents at one
    wavenumber are R-orthogonal, eq. (6))."""
    na = np.sqrt(np.einsum("in,ij,jn->n", Ja, R, Ja))
    nb = np.sqrt(np.einsum("in,ij,jn->n", Jb, R, Jb))
    return np.abs(Ja.T @ R @ Jb) / np.outer(na, nb)


def track_by_correlation(Ja, Jb, R):
    """Correspondence of the modes at one wavenumber (columns of Ja) with
    those at the next (columns of Jb): the permutation p maximising the sum of
    modal correlations C[a, p[a]] (R taken at the second wavenumber), found by
    trying every permutation (a handful of modes).  Returns (p, C[a, p[a]])."""
    from itertools import permutations
    C = modal_correlation(Ja, Jb, R)
    n = C.shape[0]
    best, best_s = None, -1.0
    for p in permutations(range(C.shape[1]), n):
        s = sum(C[a, p[a]] for a in range(n))
        if s > best_s:
            best, best_s = p, s
    p = np.array(best)
    return p, C[np.arange(n), p]
