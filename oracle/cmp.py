"""Calderon multiplicative preconditioner (section IV, eqs. (25)-(27)), dense.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
library imports or runs this module.

The preconditioned system of eq. (25) is  Z~ G^-1 Z x = Z~ G^-1 u  with

* Z   the EFIE matrix on the RWG functions f_i of the mesh (``efie``);
* Z~  the same operator tested and expanded with Buffa-Christiansen (BC)
      functions f~_i, one per RWG (eq. (26));
* G   the mixed Gram matrix G_ij = <n x f_i, f~_j> (eq. (27)).

The paper names the BC functions without defining them; this module builds
them on the barycentric refinement of the mesh (every triangle split into six
by its edge midpoints and its centroid) from their defining properties, for
closed surfaces (every vertex interior):

* the dual cell C(v) of a primal vertex v is the fan of the 2 N_v small
  triangles that touch v (N_v primal triangles around v);
* f~_e belongs to the primal edge e = (v_s, v_t): it is div-conforming on the
  refined mesh, carries a total flux l_e (the RWG's own flux) out of C(v_s)
  into C(v_t) across the dual edge (centroid of T+ -> midpoint of e ->
  centroid of T-), half across each of the two refined edges of that dual
  edge, and no flux across any other boundary edge of C(v_s) U C(v_t);
* its charge is uniform per small triangle: +l_e / (2 N_s) on each small
  triangle of C(v_s), -l_e / (2 N_t) on each of C(v_t);
* of the one-parameter family of circulations around v_s (and v_t) that
  these leave free, the flux across the refined edge from v_s (v_t) to the
  midpoint of e is zero.

Walking the fan of v from that refined edge, the flux across the j-th
radiating refined edge (j = 1 .. 2N-1) is then (j - N) l_e / (2N) in the
direction of the walk (charges 1/(2N) each, 1/2 out through each half of the
dual edge); the sink cell takes the negated pattern.  The direction v_s -> v_t
is the one of n x f_e (n the outward normal of T+), so that G has a positive
diagonal.

Everything is expressed on the refined mesh's "half functions"
h_{t,a}(r) = (r - w_a) / (2 A_t) on small triangle t (w_a its vertex a), each
carrying unit flux out of t through the edge opposite w_a: a piecewise-linear
div-conforming field is sum_{t,a} phi_{t,a} h_{t,a} with phi_{t,a} its outward
flux through that edge.  Z~ = B H B^T with B the BC flux table and H the
EFIE matrix between half functions of the refined mesh (``efie.dense_H``).
"""
import numpy as np
import scipy.sparse as sp

from .efie import ETA0, Geometry, _hf_block, dense_H, dense_Z, pair_blocks
from .quadrature import BARY, WEIGHTS
from .rwg import MeshError, build_rwg


def barycentric_refine(V, F):
    """Barycentric refinement: vertices = primal vertices, then one midpoint
    per primal edge (edges sorted by (smaller, larger) vertex), then one
    centroid per primal triangle.  Primal triangle t = (v0, v1, v2) becomes
    small triangles 6t + s, s = 0..5:
    (v0, m01, c), (m01, v1, c), (v1, m12, c), (m12, v2, c), (v2, m20, c),
    (m20, v0, c), with the orientation of t.  Returns (Vr, Fr, edges) with
    edges the (ne, 2) sorted primal edge list (midpoint of edge i is vertex
    nv + i)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    nv, nt = V.shape[0], F.shape[0]
    pairs = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    key = np.sort(pairs, axis=1)
    edges, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    ne = edges.shape[0]
    m01, m12, m20 = nv + inv[:nt], nv + inv[nt:2 * nt], nv + inv[2 * nt:]
    c = nv + ne + np.arange(nt)
    Vr = np.concatenate([V, 0.5 * (V[edges[:, 0]] + V[edges[:, 1]]), V[F].mean(axis=1)], axis=0)
    v0, v1, v2 = F[:, 0], F[:, 1], F[:, 2]
    Fr = np.stack([np.stack([v0, m01, c], 1), np.stack([m01, v1, c], 1), np.stack([v1, m12, c], 1),
                   np.stack([m12, v2, c], 1), np.stack([v2, m20, c], 1), np.stack([m20, v0, c], 1)],
                  axis=1).reshape(-1, 3)
    return Vr, Fr, edges


def _tri_normal(tv):
    n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
    return n / np.linalg.norm(n)


def bc_table(V, F):
    """BC functions of every RWG of (V, F) as a sparse (N, 3 nT_ref) table of
    half-function fluxes phi_{t,a} on the barycentric refinement (column
    3 t + a).  Returns (B, Vr, Fr)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    rwg = build_rwg(V, F)
    Vr, Fr, edges = barycentric_refine(V, F)
    nv = V.shape[0]
    ne = edges.shape[0]
    ntr = Fr.shape[0]
    # small triangles around each primal vertex
    around = [[] for _ in range(nv)]
    for t in range(ntr):
        for a in range(3):
            if Fr[t, a] < nv:
                around[Fr[t, a]].append(t)
    mid_of = {(int(a), int(b)): nv + i for i, (a, b) in enumerate(edges)}
    rows, cols, vals = [], [], []

    def local(t, w):
        """local index of refined vertex w in small triangle t"""
        return int(np.flatnonzero(Fr[t] == w)[0])

    def fan(v, m):
        """Small triangles around primal vertex v in cyclic order, starting
        with a triangle holding the refined edge (v, m), and the radiating
        vertex shared by consecutive triangles: tri[j] and tri[j-1] share the
        edge (v, rad[j]); rad[0] = m."""
        tris = around[v]
        if len(tris) < 4 or len(tris) % 2:
            raise MeshError(f"vertex {v} is not interior (open surfaces have no BC functions here)")
        start = [t for t in tris if m in Fr[t]]
        if len(start) != 2:
            raise MeshError(f"vertex {v}: the fan is not a closed disc")
        order, rad = [start[0]], [m]
        t = start[0]
        prev = m
        while True:
            # the other radiating vertex of t (neither v nor prev)
            others = [w for w in Fr[t] if w != v and w != prev]
            nxt_w = others[0]
            nb = [s for s in tris if s != t and nxt_w in Fr[s]]
            if len(nb) != 1:
                raise MeshError(f"vertex {v}: the fan is not a closed disc")
            s = nb[0]
            if s == start[0]:
                break
            order.append(s)
            rad.append(nxt_w)
            prev = nxt_w
            t = s
            if len(order) > len(tris):
                raise MeshError(f"vertex {v}: the fan is not a closed disc")
        if len(order) != len(tris):
            raise MeshError(f"vertex {v}: the fan is not a closed disc")
        return order, rad

    for e in range(rwg["N"]):
        a, b = (int(x) for x in rwg["edge"][e])
        m = mid_of[(a, b)]
        le = rwg["length"][e]
        tp = rwg["tri"][e, 0]
        n = _tri_normal(V[F[tp]])
        pp = V[rwg["free"][e, 0]]
        d = 0.5 * (V[a] + V[b]) - pp                 # across e from T+ towards T-
        s_dir = np.dot(V[b] - V[a], np.cross(n, d))
        vs, vt = (a, b) if s_dir > 0 else (b, a)
        for v, sign in ((vs, 1.0), (vt, -1.0)):
            tris, rad = fan(v, m)
            N2 = len(tris)
            Nv = N2 // 2
            for j, t in enumerate(tris):
                # flux into t across its edge (v, rad[j]) from the previous
                # triangle, and out of t across (v, rad[j+1]) into the next
                phi_in = 0.0 if j == 0 else (j - Nv) / N2
                phi_out = 0.0 if j == N2 - 1 else (j + 1 - Nv) / N2
                # edge (v, rad[j]) is opposite the third vertex of t (the centroid or midpoint not on it)
                w_in = [w for w in Fr[t] if w != v and w != rad[j]][0]
                w_out_edge = rad[j + 1] if j + 1 < N2 else rad[0]
                w_out = [w for w in Fr[t] if w != v and w != w_out_edge][0]
                flux = {local(t, w_in): -phi_in, local(t, w_out): phi_out}
                # rim edges on the dual edge of e (opposite v): half the flux each
                if j == 0 or j == N2 - 1:
                    flux[local(t, v)] = 0.5
                for loc_a, f in flux.items():
                    if f != 0.0:
                        rows.append(e)
                        cols.append(3 * t + loc_a)
                        vals.append(sign * le * f)
    B = sp.csr_matrix((vals, (rows, cols)), shape=(rwg["N"], 3 * ntr))
    B.sum_duplicates()
    return B, Vr, Fr


def _half_values(Vr, Fr, t, pts):
    """Values of the three half functions of small triangle t at pts (P, 3)
    -> (3, P, 3)."""
    tv = Vr[Fr[t]]
    A = 0.5 * np.linalg.norm(np.cross(tv[1] - tv[0], tv[2] - tv[0]))
    return (pts[None, :, :] - tv[:, None, :]) / (2 * A)


def bc_eval(B, Vr, Fr, j, t, pts):
    """Value of BC function j at points pts of small triangle t."""
    row = B.getrow(j)
    out = np.zeros((pts.shape[0], 3))
    hv = _half_values(Vr, Fr, t, pts)
    for c, v in zip(row.indices, row.data):
        if c // 3 == t:
            out += v * hv[c % 3]
    return out


def gram(V, F, B=None, Vr=None, Fr=None):
    """G_ij = <n x f_i, f~_j> (eq. (27)) by the 7-point rule on the small
    triangles (the integrand is quadratic there, so the rule is exact)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    rwg = build_rwg(V, F)
    if B is None:
        B, Vr, Fr = bc_table(V, F)
    N = rwg["N"]
    ntr = Fr.shape[0]
    G = np.zeros((N, N))
    tvs = Vr[Fr]                                             # (ntr, 3, 3)
    qp = np.einsum("qa,tax->tqx", BARY, tvs)                 # (ntr, 7, 3)
    area = 0.5 * np.linalg.norm(np.cross(tvs[:, 1] - tvs[:, 0], tvs[:, 2] - tvs[:, 0]), axis=1)
    qw = area[:, None] * WEIGHTS[None, :]
    hv = (qp[:, None, :, :] - tvs[:, :, None, :]) / (2 * area[:, None, None, None])   # (ntr, 3a, 7, 3)
    Bc = B.tocsc()
    for i in range(N):
        for side, sgn in ((0, 1.0), (1, -1.0)):
            T = rwg["tri"][i, side]
            p = V[rwg["free"][i, side]]
            nrm = _tri_normal(V[F[T]])
            Ap = rwg["area"][T]
            for s in range(6):
                t = 6 * T + s
                fi = sgn * rwg["length"][i] / (2 * Ap) * (qp[t] - p)          # (7, 3)
                nf = np.cross(nrm[None, :], fi)
                for a in range(3):
                    col = Bc.getcol(3 * t + a)
                    if col.nnz == 0:
                        continue
                    val = np.sum(qw[t] * np.einsum("qx,qx->q", nf, hv[t, a]))
                    for j, bv in zip(col.indices, col.data):
                        G[i, j] += bv * val
    return G


def dense_Ztilde(V, F, k, eta=ETA0, B=None, Vr=None, Fr=None):
    """Z~ of eq. (26): the EFIE matrix between BC functions, B H_ref B^T."""
    if B is None:
        B, Vr, Fr = bc_table(V, F)
    H = dense_H(Vr, Fr, k, eta)
    return np.asarray(B @ (B @ H.T).T)


def cmp_matrices(V, F, k, eta=ETA0):
    """(Z, Z~, G) on (V, F) at wavenumber k."""
    B, Vr, Fr = bc_table(V, F)
    return dense_Z(V, F, k, eta), dense_Ztilde(V, F, k, eta, B, Vr, Fr), gram(V, F, B, Vr, Fr)


def cmp_operator(Z, Zt, G):
    """The preconditioned matrix Z~ G^-1 Z of eq. (25)."""
    return Zt @ np.linalg.solve(G, Z)


def ztilde_rows(V, F, k, rows, X, eta=ETA0, B=None, Vr=None, Fr=None):
    """Rows `rows` of Z~ X (X: (N, ncol)) without the dense Z~: row i is
    B[i] H (B^T X) with the rows of the symmetrised half-function matrix
    0.5 (H + H^T) of the small triangles in the support of BC function i
    (the definition of ``dense_Ztilde`` restricted to those rows)."""
    if B is None:
        B, Vr, Fr = bc_table(V, F)
    X = np.asarray(X).reshape(B.shape[0], -1)
    geo = Geometry(Vr, Fr)
    ntr = Fr.shape[0]
    Y = np.asarray(B.T @ X).reshape(ntr, 3, -1)              # half-function coefficients
    Bc = B.tocsr()
    allT = np.arange(ntr)
    out = np.zeros((len(rows), X.shape[1]), dtype=np.complex128)
    for r, i in enumerate(rows):
        row = Bc.getrow(int(i))
        for t in np.unique(row.indices // 3):
            To = np.full(ntr, t)
            s1 = pair_blocks(k, geo, To, allT)
            h1 = _hf_block(k, eta, geo, To, allT, s1[0], s1[1])       # H[(t,a),(s,b)] as (s, a, b)
            s2 = pair_blocks(k, geo, allT, To)
            h2 = _hf_block(k, eta, geo, allT, To, s2[0], s2[1])       # H[(s,b),(t,a)] as (s, b, a)
            Hr = 0.5 * (h1 + h2.transpose(0, 2, 1))                    # (s, a, b)
            HY = np.einsum("sab,sbc->ac", Hr, Y)                       # (3a, ncol)
            for a in range(3):
                c = 3 * t + a
                w = row[0, c]
                if w != 0:
                    out[r] += w * HY[a]
    return out
