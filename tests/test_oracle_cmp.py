"""Pins of the oracle's Calderon preconditioner (section IV, eqs. (25)-(27)).

The paper names the Buffa-Christiansen (BC) functions and the mixed Gram
matrix but defines neither; the pins check the oracle against what the
mathematics fixes:

* the barycentric refinement: six small triangles of equal area per
  triangle, with the parent's orientation;
* every BC function, evaluated from its half-function table by its geometry
  (fields at edge quadrature points, not the table's bookkeeping), is
  div-conforming (normal flux continuous across every refined edge), has the
  uniform charges +-l/(2N) on the small triangles of its two dual cells and
  none elsewhere, carries l/2 across each half of its dual edge and nothing
  across the refined edges from its two vertices to the edge midpoint;
* the mixed Gram matrix is well conditioned, independently of the mesh size;
* the Calderon identity: with T = n x E the EFIE operator, T o T = -1/4 + K^2
  with K^2 compact, so the spectrum of G^-T Z~ G^-1 Z (the composition read
  back into RWG coefficients through the transposed Gram, whose transposition
  contributes a factor -1) clusters at +(4 pi eta)^2 / 4 (the oracle's kernel
  exp(-ikR)/R lacks the 1/(4 pi) in both Z and Z~), and Z~ G^-1 Z stays well
  conditioned where Z is not.  A wrong circulation or flux split in the BC
  functions breaks the clustering (checked by hand while writing these
  pins: condition numbers 3.5 and 129 instead of 2.2).
"""
import numpy as np
import pytest

import workloads
from oracle import cmp, efie
from oracle.rwg import MeshError, build_rwg


@pytest.fixture(scope="module")
def ico1():
    V, F = workloads.icosphere(1, 1.0)
    B, Vr, Fr = cmp.bc_table(V, F)
    return V, F, B, Vr, Fr


def _area(tv):
    return 0.5 * np.linalg.norm(np.cross(tv[..., 1, :] - tv[..., 0, :], tv[..., 2, :] - tv[..., 0, :]), axis=-1)


def test_barycentric_refinement_geometry():
    V, F = workloads.icosphere(1, 1.0)
    Vr, Fr, edges = cmp.barycentric_refine(V, F)
    nv, nt, ne = V.shape[0], F.shape[0], edges.shape[0]
    assert Vr.shape[0] == nv + ne + nt and Fr.shape[0] == 6 * nt
    a_small = _area(Vr[Fr]).reshape(nt, 6)
    a_par = _area(V[F])
    np.testing.assert_allclose(a_small, np.repeat(a_par[:, None] / 6, 6, axis=1), rtol=1e-12)
    n_par = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    tvr = Vr[Fr]
    n_sm = np.cross(tvr[:, 1] - tvr[:, 0], tvr[:, 2] - tvr[:, 0]).reshape(nt, 6, 3)
    assert np.all(np.einsum("tx,tsx->ts", n_par, n_sm) > 0)


def _edge_fluxes(B, Vr, Fr, j):
    """Outward normal flux of BC function j through every edge of every small
    triangle of its support, from the field at two Gauss points per edge:
    dict (t, local vertex opposite the edge) -> flux."""
    row = B.getrow(j)
    tris = sorted(set(int(c) // 3 for c in row.indices))
    g = 0.5 / np.sqrt(3.0)
    out = {}
    for t in tris:
        tv = Vr[Fr[t]]
        n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
        n /= np.linalg.norm(n)
        c = tv.mean(axis=0)
        for a in range(3):
            p, q = tv[(a + 1) % 3], tv[(a + 2) % 3]
            pts = np.stack([0.5 * (p + q) + s * (q - p) for s in (-g, g)])
            nu = np.cross(q - p, n)
            nu /= np.linalg.norm(nu)
            if np.dot(nu, 0.5 * (p + q) - c) < 0:
                nu = -nu
            f = cmp.bc_eval(B, Vr, Fr, j, t, pts)
            out[(t, a)] = 0.5 * np.linalg.norm(q - p) * float(np.sum(f @ nu))
    return out


def _refined_edge_map(Fr):
    m = {}
    for t in range(Fr.shape[0]):
        for a in range(3):
            key = tuple(sorted((int(Fr[t, (a + 1) % 3]), int(Fr[t, (a + 2) % 3]))))
            m.setdefault(key, []).append((t, a))
    return m


def test_bc_functions_div_conforming_uniform_charges(ico1):
    V, F, B, Vr, Fr = ico1
    rwg = build_rwg(V, F)
    nv = V.shape[0]
    emap = _refined_edge_map(Fr)
    _, _, edges = cmp.barycentric_refine(V, F)
    mid = {tuple(e): nv + i for i, e in enumerate(edges.tolist())}
    # small triangles per primal vertex
    around = {}
    for t in range(Fr.shape[0]):
        for w in Fr[t]:
            if w < nv:
                around.setdefault(int(w), set()).add(t)
    for j in range(rwg["N"]):
        fl = _edge_fluxes(B, Vr, Fr, j)
        le = rwg["length"][j]
        a, b = (int(x) for x in rwg["edge"][j])
        m = mid[(a, b)]
        # continuity: outflow of one side = inflow of the other (zero field outside the support)
        for key, sides in emap.items():
            f = [fl.get(s, 0.0) for s in sides]
            if len(sides) == 2:
                assert abs(f[0] + f[1]) < 1e-12 * le, (j, key, f)
        charge = {}
        for (t, loc), f in fl.items():
            charge[t] = charge.get(t, 0.0) + f
        ca, cb = around[a], around[b]
        sa = sum(charge.get(t, 0.0) for t in ca)
        vs, vt = (a, b) if sa > 0 else (b, a)
        for t, q in charge.items():
            if t in around[vs]:
                assert abs(q - le / len(around[vs])) < 1e-12 * le, (j, t, q)
            elif t in around[vt]:
                assert abs(q + le / len(around[vt])) < 1e-12 * le, (j, t, q)
            else:
                assert abs(q) < 1e-12 * le, (j, t, q)
        # no flux across the refined edges from the two vertices to the midpoint
        for v in (vs, vt):
            for (t, loc) in emap[tuple(sorted((v, m)))]:
                assert abs(fl.get((t, loc), 0.0)) < 1e-12 * le
        # half of the flux across each half of the dual edge, from C(vs) into C(vt)
        c_p, c_m = (Vr.shape[0] - F.shape[0] + int(rwg["tri"][j, s]) for s in (0, 1))
        for c in (c_p, c_m):
            sides = emap[tuple(sorted((m, c)))]
            t_s = [s for s in sides if s[0] in around[vs]]
            assert len(t_s) == 1 and abs(fl[t_s[0]] - 0.5 * le) < 1e-12 * le


def test_gram_well_conditioned_mesh_independent(ico1):
    V, F, B, Vr, Fr = ico1
    G1 = cmp.gram(V, F, B, Vr, Fr)
    V2, F2 = workloads.icosphere(2, 1.0)
    G2 = cmp.gram(V2, F2)
    c1, c2 = np.linalg.cond(G1), np.linalg.cond(G2)
    assert np.all(np.diag(G1) > 0) and np.all(np.diag(G2) > 0)
    assert c1 < 4 and c2 < 4 and abs(c2 / c1 - 1) < 0.2, (c1, c2)


def test_calderon_identity_clusters_spectrum(ico1):
    V, F, B, Vr, Fr = ico1
    k = 0.5
    Z = efie.dense_Z(V, F, k)
    Zt = cmp.dense_Ztilde(V, F, k, B=B, Vr=Vr, Fr=Fr)
    G = cmp.gram(V, F, B, Vr, Fr)
    A = cmp.cmp_operator(Z, Zt, G)
    assert np.linalg.cond(Z) > 100
    assert np.linalg.cond(A) < 3
    M = np.linalg.solve(G.T, A)
    r = np.linalg.eigvals(M) / ((4 * np.pi * efie.ETA0) ** 2 / 4)
    assert np.mean(np.abs(r - 1) < 0.25) >= 0.95
    # Z~ is the EFIE between BC functions: complex symmetric like Z
    assert np.abs(Zt - Zt.T).max() < 1e-10 * np.abs(Zt).max()


def test_open_surface_has_no_bc_functions():
    V, F = workloads.plate(4, 4, 0.1)
    with pytest.raises(MeshError):
        cmp.bc_table(V, F)


def test_ztilde_rows_equal_dense_rows(ico1):
    """The row-wise product (used for large meshes) is the dense definition."""
    V, F, B, Vr, Fr = ico1
    k = 0.5
    Zt = cmp.dense_Ztilde(V, F, k, B=B, Vr=Vr, Fr=Fr)
    X = workloads.cn01_block(B.shape[0], 2, 3)
    rows = [0, 5, 77, 119]
    zr = cmp.ztilde_rows(V, F, k, rows, X, B=B, Vr=Vr, Fr=Fr)
    ref = (Zt @ X)[rows]
    assert np.abs(zr - ref).max() < 1e-13 * np.abs(ref).max()
