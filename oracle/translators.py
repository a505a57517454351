"""Truncated translators and the point test of the numerical-results section,
in the paper's own time convention (Green's function exp(ikR)/R, eq. (3)).

  alpha   (eq. (10)) = sum_{l<=L} i^l (2l+1) h_l^(1)(k r) P_l(khat.rhat)
  alpha_S (eq. (16)) = i sum i^l (2l+1) y_l(k r) P_l(khat.rhat)
  alpha_R (eq. (20)) = -i sum i^l (2l+1) j_l(k r) P_l(khat.rhat)

and each kernel K(r_ij) in {exp(ikr)/r, cos(kr)/r, sin(kr)/r} is

  (ik/4 pi) int d^2khat exp(ik khat.(r_im + r_m'j)) alpha_*(khat, r_mm')     (eqs. (9), (15), (19))

with the sphere integral on Gauss-Legendre (L+1) x uniform 2(L+1) samples and
L from the truncation rule of eq. (30), L = ceil(kd + 1.8 d0^(2/3) (kd)^(1/3)),
d = sqrt(3) a.
"""
import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn

from .planewave import sphere_sampling


def truncation_L(k: float, a: float, d0: float = 3.0) -> int:
    kd = k * np.sqrt(3.0) * a
    return int(np.ceil(kd + 1.8 * d0 ** (2.0 / 3.0) * kd ** (1.0 / 3.0)))


def translator(kind: str, L: int, k: float, X: np.ndarray, khat: np.ndarray) -> np.ndarray:
    r = np.linalg.norm(X)
    c = khat @ (X / r)
    out = np.zeros(khat.shape[0], dtype=np.complex128)
    for l in range(L + 1):
        if kind == "h":
            z = spherical_jn(l, k * r) + 1j * spherical_yn(l, k * r)
            pre = 1.0
        elif kind == "y":
            z = spherical_yn(l, k * r)
            pre = 1j
        elif kind == "j":
            z = spherical_jn(l, k * r)
            pre = -1j
        else:
            raise ValueError(kind)
        out += pre * (1j ** l) * (2 * l + 1) * z * eval_legendre(l, c)
    return out


def expansion(kind: str, k: float, a: float, ri, rm, rmp, rj, d0: float = 3.0):
    """Right-hand side of eq. (9)/(15)/(19) for the given points and centres."""
    L = truncation_L(k, a, d0)
    khat, w = sphere_sampling(L)
    d = (np.asarray(ri) - rm) + (np.asarray(rmp) - rj)
    alpha = translator(kind, L, k, np.asarray(rm) - np.asarray(rmp), khat)
    return (1j * k / (4 * np.pi)) * np.sum(w * np.exp(1j * k * (khat @ d)) * alpha)


def closed_form(kind: str, k: float, r: float):
    return {"h": np.exp(1j * k * r) / r, "y": np.cos(k * r) / r, "j": np.sin(k * r) / r}[kind]


def point_test(kind: str, case: int, a_over_lambda: float, d0: float = 3.0):
    """Relative error of the plane-wave expansion at the paper's two point
    configurations (box size a, wavelength 1)."""
    a = a_over_lambda
    k = 2 * np.pi
    rj = np.array([0.9999 * a, 1.0 * a, 0.0])
    rmp = np.array([0.5 * a, 0.5 * a, 0.5 * a])
    if case == 1:
        ri = np.array([2.9999 * a, 0.0, 1.0 * a])
        rm = np.array([2.5 * a, 0.5 * a, 0.5 * a])
    else:
        ri = np.array([1.0001 * a, 0.0, 0.0])
        rm = np.array([1.5 * a, 0.5 * a, 0.5 * a])
    rhs = expansion(kind, k, a, ri, rm, rmp, rj, d0)
    lhs = closed_form(kind, k, np.linalg.norm(ri - rj))
    return abs(rhs - lhs) / abs(lhs), rhs, lhs
