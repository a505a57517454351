"""Galerkin EFIE impedance matrix on RWG functions (eq. (5)), plain definition.

Public convention (see package docstring):

  Z_mn = ik eta sum_{T in m} sum_{T' in n} int_T int_T'
           [ f_m(r).f_n(r') - (1/k^2) div f_m div' f_n ] exp(-ikR)/R  dS' dS

(the mixed-potential form of <f, [I - grad grad'/k^2] g, f> after integrating
the grad grad' term by parts), so R = Re Z = k eta <..sin(kR)/R..> and
X = Im Z = k eta <..cos(kR)/R..> as in eqs. (17) and (21) up to the overall
sign of R.

Discretisation (the same definition the GPU fill implements independently):

* outer integral: 7-point rule on T; inner integral: 7-point rule on T';
* for a "near-singular" triangle pair, |c_T - c_T'|^2 < (1.5 max(h_T, h_T'))^2
  with c the centroid and h the longest edge, the inner integral of the 1/R
  part is done in closed form (``potentials``) and the remainder
  (exp(-ikR) - 1)/R by the 7-point rule (limit -ik at R = 0);
* a near-singular pair's block is averaged with the transposed block computed
  with the roles of the two triangles exchanged, so Z = Z^T.  (For the other
  pairs the double 7 x 7 sum is already symmetric.)

The k-derivative follows from Z = i eta [k A - B/k] with A = <f.f' G>,
B = <div f div' f' G>, dG/dk = -i exp(-ikR):

  dZ/dk = i eta <[f.f' + div div'/k^2] G> + eta <[k f.f' - div div'/k] exp(-ikR)>

whose second bracket is smooth (no extraction).
"""
import numpy as np

from .quadrature import WEIGHTS, tri_points
from .potentials import potential_integrals
from .rwg import build_rwg

ETA0 = 376.730313668


class Geometry:
    def __init__(self, V, F):
        V = np.asarray(V, dtype=np.float64)
        F = np.asarray(F, dtype=np.int64)
        self.tv = V[F]                                       # (T, 3, 3)
        e1 = self.tv[:, 1] - self.tv[:, 0]
        e2 = self.tv[:, 2] - self.tv[:, 0]
        cr = np.cross(e1, e2)
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / (2 * self.area[:, None])
        self.centroid = self.tv.mean(axis=1)
        el = np.stack([np.linalg.norm(self.tv[:, (i + 1) % 3] - self.tv[:, i], axis=1) for i in range(3)], 1)
        self.hmax = el.max(axis=1)
        self.qp = tri_points(self.tv)                        # (T, 7, 3)
        self.qw = self.area[:, None] * WEIGHTS[None, :]      # (T, 7)


def near_singular(geo: Geometry, To, Ts):
    dc = geo.centroid[To] - geo.centroid[Ts]
    h = np.maximum(geo.hmax[To], geo.hmax[Ts])
    return np.einsum("px,px->p", dc, dc) < (1.5 * h) ** 2


def _gm1_over_r(k, R):
    """(exp(-ikR) - 1)/R, with its limit -ik at R = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (-2.0 * np.sin(0.5 * k * R) ** 2 - 1j * np.sin(k * R)) / R
    return np.where(R > 0, v, -1j * k)


def pair_blocks(k, geo: Geometry, To, Ts, deriv=False):
    """Triangle-pair integrals, outer integral on To[p], inner on Ts[p]:

      S0[p]      = int int G
      Sv[p,a,b]  = int int (r - v_a).(r' - v'_b) G
      (deriv)  E0, Ev = the same with exp(-ikR) in place of G = exp(-ikR)/R
    """
    To = np.asarray(To)
    Ts = np.asarray(Ts)
    P = To.size
    ro = geo.qp[To]                    # (P, 7, 3)
    rs = geo.qp[Ts]
    wo = geo.qw[To]                    # (P, 7)
    ws = geo.qw[Ts]
    Ua = ro[:, :, None, :] - geo.tv[To][:, None, :, :]      # (P, 7, 3a, 3x)
    Ub = rs[:, :, None, :] - geo.tv[Ts][:, None, :, :]      # (P, 7, 3b, 3x)
    Rv = ro[:, :, None, :] - rs[:, None, :, :]
    R = np.linalg.norm(Rv, axis=3)                          # (P, 7, 7)
    sing = near_singular(geo, To, Ts)
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.where(R > 0, np.exp(-1j * k * R) / np.where(R > 0, R, 1.0), 0.0)
    G = np.where(sing[:, None, None], _gm1_over_r(k, R), G)   # regular part only for singular pairs
    WW = wo[:, :, None] * ws[:, None, :]

    def contract(K):
        WK = WW * K
        S0 = WK.sum(axis=(1, 2))
        M1 = np.matmul(WK, Ub.reshape(P, 7, 9)).reshape(P, 7, 3, 3)
        Sv = np.einsum("Ppax,Ppbx->Pab", Ua, M1)
        return S0, Sv

    S0, Sv = contract(G)
    idx = np.flatnonzero(sing)
    if idx.size:
        # closed-form inner integral of the 1/R part at every outer point
        tvs = geo.tv[Ts[idx]]                                # (Q, 3, 3)
        rq = ro[idx].reshape(-1, 3)
        tvq = np.repeat(tvs, 7, axis=0)
        I1, Iv = potential_integrals(rq, tvq)
        I1 = I1.reshape(-1, 7)
        Iv = Iv.reshape(-1, 7, 3)
        n = geo.normal[Ts[idx]]
        d = np.einsum("qpx,qx->qp", ro[idx] - tvs[:, None, 0, :], n)
        # int (r' - v'_b)/R = int (r' - r)/R + (r - v'_b) int 1/R, and r' - r = (rho' - rho) - d n
        rel = Iv - (d * I1)[:, :, None] * n[:, None, :]       # (Q, 7, 3)
        inner = rel[:, :, None, :] + (ro[idx][:, :, None, :] - tvs[:, None, :, :]) * I1[:, :, None, None]
        wq = wo[idx]
        S0[idx] += np.einsum("qp,qp->q", wq, I1)
        Sv[idx] += np.einsum("qp,qpax,qpbx->qab", wq, Ua[idx], inner)
    if not deriv:
        return S0, Sv, sing
    E = np.exp(-1j * k * R)
    E0, Ev = contract(E)
    return S0, Sv, E0, Ev, sing


def _hf_block(k, eta, geo, To, Ts, S0, Sv):
    """ik eta [Sv/(4 A A') - S0/(k^2 A A')] per half-function pair (without s l factors)."""
    AA = (geo.area[To] * geo.area[Ts])[:, None, None]
    return 1j * k * eta * (Sv / (4 * AA) - S0[:, None, None] / (k * k * AA))


def _hf_dblock(k, eta, geo, To, Ts, S0, Sv, E0, Ev):
    AA = (geo.area[To] * geo.area[Ts])[:, None, None]
    t1 = 1j * eta * (Sv / (4 * AA) + S0[:, None, None] / (k * k * AA))
    t2 = eta * (k * Ev / (4 * AA) - E0[:, None, None] / (k * AA))
    return t1 + t2


def _incidence(rwg, nT):
    """(N, 3 nT) matrix with s*l at (rwg, 3T+a) for each half function."""
    import scipy.sparse as sp
    hr = rwg["hf_rwg"].ravel()
    hs = rwg["hf_sign"].ravel()
    cols = np.flatnonzero(hr >= 0)
    rows = hr[cols]
    vals = hs[cols] * rwg["length"][rows]
    return sp.csr_matrix((vals, (rows, cols)), shape=(rwg["N"], 3 * nT))


def _dense_half(V, F, k, eta, deriv, chunk):
    """Symmetrised half-function matrices (3 nT x 3 nT), row/column 3 T + a."""
    geo = Geometry(V, F)
    nT = geo.tv.shape[0]
    H = np.zeros((nT, 3, nT, 3), dtype=np.complex128)
    dH = np.zeros_like(H) if deriv else None
    allT = np.arange(nT)
    for t0 in range(0, nT, chunk):
        obs = np.arange(t0, min(nT, t0 + chunk))
        To = np.repeat(obs, nT)
        Ts = np.tile(allT, obs.size)
        out = pair_blocks(k, geo, To, Ts, deriv)
        blk = _hf_block(k, eta, geo, To, Ts, out[0], out[1])
        H[obs] = blk.reshape(obs.size, nT, 3, 3).transpose(0, 2, 1, 3)
        if deriv:
            dblk = _hf_dblock(k, eta, geo, To, Ts, out[0], out[1], out[2], out[3])
            dH[obs] = dblk.reshape(obs.size, nT, 3, 3).transpose(0, 2, 1, 3)

    def sym(Hm):
        Hm = Hm.reshape(3 * nT, 3 * nT)
        return 0.5 * (Hm + Hm.T)              # only near-singular blocks change
    return (sym(H), sym(dH)) if deriv else (sym(H),)


def dense_H(V, F, k, eta=ETA0, chunk=48):
    """EFIE matrix between the half functions h_{T,a}(r) = (r - v_a)/(2 A_T)
    of every triangle (unit flux out of T through the edge opposite v_a),
    row/column 3 T + a: Z = P H P^T with P the incidence of RWGs on half
    functions (sign times edge length)."""
    return _dense_half(V, F, k, eta, False, chunk)[0]


def dense_Z(V, F, k, eta=ETA0, deriv=False, chunk=48):
    """Dense Z (N x N complex128); with deriv=True returns (Z, dZ/dk)."""
    rwg = build_rwg(V, F)
    Hs = _dense_half(V, F, k, eta, deriv, chunk)
    P = _incidence(rwg, np.asarray(F).shape[0])
    Zs = [np.asarray(P @ (P @ Hm.T).T) for Hm in Hs]
    return (Zs[0], Zs[1]) if deriv else Zs[0]


def rows_Z(V, F, k, rows, eta=ETA0, deriv=False, geo=None, rwg=None):
    """Rows of Z (len(rows) x N).  With deriv=True returns (Zrows, dZ/dk rows)."""
    geo = geo or Geometry(V, F)
    rwg = rwg or build_rwg(V, F)
    nT = geo.tv.shape[0]
    P = _incidence(rwg, nT)
    allT = np.arange(nT)
    out_rows = np.zeros((len(rows), rwg["N"]), dtype=np.complex128)
    out_d = np.zeros_like(out_rows) if deriv else None
    for i, m in enumerate(rows):
        h = np.zeros((3 * nT,), dtype=np.complex128)
        dh = np.zeros_like(h) if deriv else None
        for side in range(2):
            T = rwg["tri"][m, side]
            a = rwg["loc"][m, side]
            coef = rwg["hf_sign"][T, a] * rwg["length"][m]
            To = np.full(nT, T)
            res = pair_blocks(k, geo, To, allT, deriv)
            blk = _hf_block(k, eta, geo, To, allT, res[0], res[1])[:, a, :]      # (nT, 3b)
            if deriv:
                dblk = _hf_dblock(k, eta, geo, To, allT, *res[:4])[:, a, :]
            sing = np.flatnonzero(res[-1])
            if sing.size:
                # average near-singular blocks with the exchanged evaluation
                Ts = allT[sing]
                To2 = np.full(sing.size, T)
                res2 = pair_blocks(k, geo, Ts, To2, deriv)
                b2 = _hf_block(k, eta, geo, Ts, To2, res2[0], res2[1])[:, :, a]     # (Q, 3b)
                blk[sing] = 0.5 * (blk[sing] + b2)
                if deriv:
                    db2 = _hf_dblock(k, eta, geo, Ts, To2, *res2[:4])[:, :, a]
                    dblk[sing] = 0.5 * (dblk[sing] + db2)
            h += coef * blk.ravel()
            if deriv:
                dh += coef * dblk.ravel()
        out_rows[i] = P @ h
        if deriv:
            out_d[i] = P @ dh
    if deriv:
        return out_rows, out_d
    return out_rows
