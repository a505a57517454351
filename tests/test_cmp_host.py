"""The library's Calderon tables (host side, no GPU) against the oracle's:
the mixed Gram matrix G entry by entry, and the Buffa-Christiansen functions
as fields (the library stores them on the refined mesh's RWG functions in its
own small-triangle layout, the oracle on half functions in another; both are
evaluated at the centroid of every small triangle, matched by geometry).
Sphere of radius 0.5 wavelength, icosahedron subdivided three times (1,920
RWG), the handle built host-only."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import cmp
from oracle.rwg import build_rwg


@pytest.fixture(scope="module")
def tables():
    from paper_1412_1756_amd import Operator
    V, F = workloads.icosphere(3, 0.5)
    op = Operator(V, F, 2 * np.pi, nlv=3, host_only=True)
    info = op.cmp_build(nlv=3)
    B, Vr, Fr = cmp.bc_table(V, F)
    return V, F, op, info, B, Vr, Fr


def test_cmp_build_info(tables):
    V, F, op, info, B, Vr, Fr = tables
    assert info["N_refined"] == 6 * op.N and info["nlv_refined"] == 3
    with pytest.raises(Exception):
        op.cmp_apply(None)


def test_gram_matches_oracle(tables):
    V, F, op, info, B, Vr, Fr = tables
    ptr, col, val = op.cmp_export("G")
    Gl = sp.csr_matrix((val, col, ptr), shape=(op.N, op.N)).toarray()
    Go = cmp.gram(V, F, B, Vr, Fr)
    assert np.abs(Gl - Go).max() < 1e-12 * np.abs(Go).max()
    # the same pattern (entries that cancel to round-off aside)
    big = 1e-12 * np.abs(Go).max()
    assert ((np.abs(Gl) > big) == (np.abs(Go) > big)).all()


def _library_refinement(V, F):
    """The refined mesh in the library's documented layout."""
    rw = build_rwg(V, F)
    nv, N = V.shape[0], rw["N"]
    eid = {tuple(e): i for i, e in enumerate(rw["edge"].tolist())}
    Vl = np.concatenate([V, 0.5 * (V[rw["edge"][:, 0]] + V[rw["edge"][:, 1]]), V[F].mean(axis=1)])
    Fl = []
    for t, tri in enumerate(np.asarray(F).tolist()):
        c = nv + N + t
        for a in range(3):
            mn = nv + eid[tuple(sorted((tri[a], tri[(a + 1) % 3])))]
            mp = nv + eid[tuple(sorted((tri[(a + 2) % 3], tri[a])))]
            Fl += [(tri[a], mn, c), (tri[a], c, mp)]
    return Vl, np.array(Fl)


def test_bc_functions_match_oracle(tables):
    V, F, op, info, B, Vr, Fr = tables
    Vl, Fl = _library_refinement(V, F)
    rr = build_rwg(Vl, Fl)
    assert rr["N"] == info["N_refined"]
    ptr, col, val = op.cmp_export("B")
    Bl = sp.csr_matrix((val, col, ptr), shape=(op.N, rr["N"]))
    # library field on small triangle t: sum over refined RWGs e with t a side
    # of B[:, e] * (+-) l_e/(2A_t) (r - p_e,t)
    rows, cols, vals = [], [], []
    for e in range(rr["N"]):
        for s, sg in ((0, 1.0), (1, -1.0)):
            rows.append(e)
            cols.append(3 * rr["tri"][e, s] + rr["loc"][e, s])
            vals.append(sg * rr["length"][e])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(rr["N"], 3 * Fl.shape[0]))
    Bh = (Bl @ P).tocsc()                  # the library's BC functions on its half functions
    Bo = B.tocsc()
    key = {tuple(sorted(map(tuple, np.round(Vl[f], 12).tolist()))): i for i, f in enumerate(Fl)}
    worst, scale = 0.0, 0.0
    for t in range(Fr.shape[0]):
        tv = Vr[Fr[t]]
        tl = key[tuple(sorted(map(tuple, np.round(tv, 12).tolist())))]
        tvl = Vl[Fl[tl]]
        A = 0.5 * np.linalg.norm(np.cross(tv[1] - tv[0], tv[2] - tv[0]))
        cen = tv.mean(axis=0)
        fo = sum(Bo[:, 3 * t + a].toarray() * (cen - tv[a])[None, :] / (2 * A) for a in range(3))
        fl = sum(Bh[:, 3 * tl + a].toarray() * (cen - tvl[a])[None, :] / (2 * A) for a in range(3))
        worst = max(worst, np.abs(fo - fl).max())
        scale = max(scale, np.abs(fo).max())
    assert worst < 1e-12 * scale, (worst, scale)


def test_open_surface_rejected():
    from paper_1412_1756_amd import Operator, CmError
    V, F = workloads.plate(20, 20, 0.05)
    op = Operator(V, F, 2 * np.pi, nlv=3, host_only=True)
    with pytest.raises(CmError, match="closed surface"):
        op.cmp_build()
