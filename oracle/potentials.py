"""Closed-form potential integrals over a flat triangle.

For an observation point r and a planar triangle T' with unit normal n
(vertices counter-clockwise about n), write r = rho + d n with rho in the plane
of T'.  For each edge from vertex a to vertex b let s = (b - a)/|b - a|,
u = s x n (in-plane, pointing out of T'), l+ = (b - rho).s, l- = (a - rho).s,
P0 = (a - rho).u, R+ = |r - b|, R- = |r - a| and R0^2 = P0^2 + d^2.  Then

  int_T' 1/|r - r'| dS'
      = sum_edges { P0 ln[(R+ + l+)/(R- + l-)]
                    - |d| [atan(P0 l+ / (R0^2 + |d| R+)) - atan(P0 l- / (R0^2 + |d| R-))] }

  int_T' (rho' - rho)/|r - r'| dS'
      = 1/2 sum_edges u [ R0^2 ln[(R+ + l+)/(R- + l-)] + l+ R+ - l- R- ]

(Wilton, Rao, Glisson et al., IEEE TAP 1984; Graglia, IEEE TAP 1993).  These
extract the 1/R singularity of the Green's function (eq. (3)) from the
Galerkin integrals of eq. (5) when two triangles are close.
"""
import numpy as np


def _log_r_plus_l(R, l, R0sq):
    # ln(R + l) without cancellation: for l < 0, R + l = R0^2 / (R - l)
    with np.errstate(divide="ignore", invalid="ignore"):
        pos = np.log(np.where(l >= 0, R + l, 1.0))
        neg = np.log(np.where(l < 0, R0sq, 1.0)) - np.log(np.where(l < 0, R - l, 1.0))
    return np.where(l >= 0, pos, neg)


def potential_integrals(r: np.ndarray, tv: np.ndarray):
    """r: (M, 3) points; tv: (M, 3, 3) triangle vertices.
    Returns (I1 (M,), Iv (M, 3)) = (int 1/R dS', int (rho' - rho)/R dS')."""
    r = np.asarray(r, dtype=np.float64)
    tv = np.asarray(tv, dtype=np.float64)
    n = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    d = np.einsum("mx,mx->m", r - tv[:, 0], n)
    rho = r - d[:, None] * n
    ad = np.abs(d)
    scale2 = np.einsum("mx,mx->m", tv[:, 1] - tv[:, 0], tv[:, 1] - tv[:, 0])
    I1 = np.zeros(r.shape[0])
    Iv = np.zeros_like(r)
    for i in range(3):
        a = tv[:, i]
        b = tv[:, (i + 1) % 3]
        s = b - a
        s /= np.linalg.norm(s, axis=1, keepdims=True)
        u = np.cross(s, n)
        lp = np.einsum("mx,mx->m", b - rho, s)
        lm = np.einsum("mx,mx->m", a - rho, s)
        P0 = np.einsum("mx,mx->m", a - rho, u)
        Rp = np.linalg.norm(r - b, axis=1)
        Rm = np.linalg.norm(r - a, axis=1)
        R0sq = P0 * P0 + d * d
        degenerate = R0sq <= 1e-28 * scale2          # point on the edge's line
        R0safe = np.where(degenerate, 1.0, R0sq)
        L = _log_r_plus_l(Rp, lp, R0safe) - _log_r_plus_l(Rm, lm, R0safe)
        L = np.where(degenerate, 0.0, L)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.arctan(P0 * lp / (R0safe + ad * Rp)) - np.arctan(P0 * lm / (R0safe + ad * Rm))
        t = np.where(degenerate, 0.0, t)
        I1 += P0 * L - ad * t
        Iv += 0.5 * u * (R0sq * L + lp * Rp - lm * Rm)[:, None]
    return I1, Iv
