"""Rao-Wilton-Glisson basis functions on a triangle mesh (eq. (4)).

One basis function per edge shared by exactly two triangles.  Order: interior
edges sorted by (smaller vertex index, larger vertex index).  T+ is the
lower-numbered of the two triangles, T- the other; p+ and p- are the vertices
of T+ and T- opposite the edge.  With edge length l and triangle area A,

  f(r) = l / (2 A+) (r - p+)   on T+,     div f = +l / A+
  f(r) = l / (2 A-) (p- - r)   on T-,     div f = -l / A-

A "half function" is the restriction of f to one triangle; on triangle T it is
identified by the local vertex a (0, 1, 2) opposite its edge.
"""
import numpy as np


class MeshError(ValueError):
    pass


def build_rwg(V: np.ndarray, F: np.ndarray) -> dict:
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    nT = F.shape[0]
    if not np.all(np.isfinite(V)):
        raise MeshError("non-finite vertex coordinates")
    tv = V[F]
    area = 0.5 * np.linalg.norm(np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0]), axis=1)
    if np.any(area <= 0.0):
        raise MeshError("degenerate (zero-area) triangle")
    # local vertex a of triangle t is opposite the edge (F[t,a+1], F[t,a+2])
    ea = F[:, [1, 2, 0]]
    eb = F[:, [2, 0, 1]]
    lo = np.minimum(ea, eb).ravel()
    hi = np.maximum(ea, eb).ravel()
    tri = np.repeat(np.arange(nT), 3)
    loc = np.tile(np.arange(3), nT)
    order = np.lexsort((tri, hi, lo))
    lo, hi, tri, loc = lo[order], hi[order], tri[order], loc[order]
    newkey = np.ones(lo.size, dtype=bool)
    newkey[1:] = (lo[1:] != lo[:-1]) | (hi[1:] != hi[:-1])
    start = np.flatnonzero(newkey)
    count = np.diff(np.append(start, lo.size))
    if np.any(count > 2):
        raise MeshError("non-manifold edge shared by more than two triangles")
    s = start[count == 2]
    N = s.size
    tp, tm = tri[s], tri[s + 1]                   # lexsort puts the lower triangle first
    ap, am = loc[s], loc[s + 1]
    edge = np.stack([lo[s], hi[s]], axis=1)
    length = np.linalg.norm(V[edge[:, 1]] - V[edge[:, 0]], axis=1)
    hf_rwg = -np.ones((nT, 3), dtype=np.int64)
    hf_sign = np.zeros((nT, 3))
    hf_rwg[tp, ap] = np.arange(N)
    hf_rwg[tm, am] = np.arange(N)
    hf_sign[tp, ap] = 1.0
    hf_sign[tm, am] = -1.0
    return dict(N=N, edge=edge, tri=np.stack([tp, tm], 1), loc=np.stack([ap, am], 1),
                free=np.stack([F[tp, ap], F[tm, am]], 1), length=length, area=area,
                hf_rwg=hf_rwg, hf_sign=hf_sign)


def rwg_eval(V, F, rwg, n, pts_on_plus, pts_on_minus):
    """Values of basis function n at points given on T+ and on T- (for tests)."""
    V = np.asarray(V, dtype=np.float64)
    tp, tm = rwg["tri"][n]
    l = rwg["length"][n]
    Ap, Am = rwg["area"][tp], rwg["area"][tm]
    pp, pm = V[rwg["free"][n, 0]], V[rwg["free"][n, 1]]
    return l / (2 * Ap) * (pts_on_plus - pp), l / (2 * Am) * (pm - pts_on_minus)
