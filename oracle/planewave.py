"""R = Re Z through the plane-wave representation of the regular kernel.

The sin(kR)/R kernel has an addition theorem with no validity restriction
(eq. (19)); in its untranslated form sin(k|r - r'|)/|r - r'| equals
(k / 4 pi) times the integral over the unit sphere of exp(ik khat.(r - r')).
With the operator [I - grad grad'/k^2] acting as the transverse projector
(I - khat khat) on each plane wave, the resistance matrix becomes

  R_mn = (k^2 eta / 4 pi) sum_q w_q  Fperp_m(khat_q) . conj(Fperp_n(khat_q)),
  F_m(khat) = sum_{T in m} sum_{points} w A f_m(r) exp(ik khat.(r - c)),

evaluated here on the same 7-point rule as the Galerkin fill, with
Gauss-Legendre sampling in cos(theta) (L+1 nodes) and 2(L+1) uniform phi
samples, L >= k r_max + 20.  This is positive semidefinite by construction
and involves no singular integral, so it pins the sign and the prefactors of R
independently of ``efie``.  (It equals the dyadic point-quadrature form; the
mixed-potential form of ``efie`` differs from it only by the quadrature error
of the integration by parts.)
"""
import numpy as np

from .efie import ETA0, Geometry
from .rwg import build_rwg


def sphere_sampling(L: int):
    x, wx = np.polynomial.legendre.leggauss(L + 1)
    th = np.arccos(x)
    nphi = 2 * (L + 1)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    khat = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    return khat, w


def radiation_vectors(V, F, k, khat, center=None):
    """F_m(khat) for every RWG m: (N, K, 3) complex."""
    geo = Geometry(V, F)
    rwg = build_rwg(V, F)
    c = np.mean(np.asarray(V, dtype=np.float64), axis=0) if center is None else center
    N = rwg["N"]
    out = np.zeros((N, khat.shape[0], 3), dtype=np.complex128)
    for side in range(2):
        T = rwg["tri"][:, side]
        a = rwg["loc"][:, side]
        s = 1.0 if side == 0 else -1.0
        coef = s * rwg["length"] / (2 * geo.area[T])                  # (N,)
        pts = geo.qp[T]                                                # (N, 7, 3)
        wts = geo.qw[T]                                                # (N, 7)
        vert = geo.tv[T, a]                                            # (N, 3)
        fv = coef[:, None, None] * (pts - vert[:, None, :])            # (N, 7, 3)
        ph = np.exp(1j * k * np.einsum("npx,qx->npq", pts - c, khat))  # (N, 7, K)
        out += np.einsum("np,npx,npq->nqx", wts, fv, ph)
    return out


def R_planewave(V, F, k, eta=ETA0, extra=20):
    V = np.asarray(V, dtype=np.float64)
    c = V.mean(axis=0)
    rmax = np.max(np.linalg.norm(V - c, axis=1))
    L = int(np.ceil(k * rmax + extra))
    khat, w = sphere_sampling(L)
    Fm = radiation_vectors(V, F, k, khat, c)
    Fp = Fm - khat[None, :, :] * np.einsum("nqx,qx->nq", Fm, khat)[:, :, None]
    A = (Fp * np.sqrt(w)[None, :, None]).reshape(Fp.shape[0], -1)
    R = (k * k * eta / (4 * np.pi)) * (A @ A.conj().T)
    return R.real, R.imag
