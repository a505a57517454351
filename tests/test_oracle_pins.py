"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign, a transposed operand, a wrong prefactor) fails it."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import workloads
from oracle import efie, modes, planewave, translators
from oracle.potentials import potential_integrals
from oracle.quadrature import BARY, WEIGHTS
from oracle.rwg import MeshError, build_rwg

K0 = 2 * np.pi
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- quadrature
def test_seven_point_rule_exact_to_degree_five():
    # int_T l1^a l2^b l3^c dA = 2 A a! b! c! / (a+b+c+2)!
    f = math.factorial
    for a in range(7):
        for b in range(7 - a):
            for c in range(7 - a - b):
                q = np.sum(WEIGHTS * BARY[:, 0] ** a * BARY[:, 1] ** b * BARY[:, 2] ** c)
                exact = 2 * f(a) * f(b) * f(c) / f(a + b + c + 2)
                if a + b + c <= 5:
                    assert abs(q - exact) < 1e-15, (a, b, c)
                elif a + b + c == 6 and max(a, b, c) == 6:
                    assert abs(q - exact) > 1e-4      # not a trivially exact rule


# ---------------------------------------------------------------- RWG
def test_rwg_counts_and_order():
    V, F = workloads.icosphere(3, 0.5)
    r = build_rwg(V, F)
    assert r["N"] == 3 * F.shape[0] // 2 == 1920
    e = r["edge"]
    assert np.all(e[:, 0] < e[:, 1])
    key = e[:, 0] * 10**6 + e[:, 1]
    assert np.all(np.diff(key) > 0)
    assert np.all(r["tri"][:, 0] < r["tri"][:, 1])
    Vp, Fp = workloads.plate(100, 100, 0.1)
    assert build_rwg(Vp, Fp)["N"] == 29800


def test_rwg_normal_flux_and_divergence():
    V, F = workloads.icosphere(2, 1.0)
    r = build_rwg(V, F)
    for n in [0, 7, 123, r["N"] - 1]:
        a, b = V[r["edge"][n, 0]], V[r["edge"][n, 1]]
        t = np.linspace(0.1, 0.9, 5)[:, None]
        pts = a + t * (b - a)
        fp, fm = efie_free = __import__("oracle.rwg", fromlist=["rwg_eval"]).rwg_eval(V, F, r, n, pts, pts)
        # unit normal flux across the edge, continuous from T+ to T-
        pp = V[r["free"][n, 0]]
        u = (pts[0] - pp) - np.dot(pts[0] - pp, (b - a)) / np.dot(b - a, b - a) * (b - a)
        u /= np.linalg.norm(u)
        np.testing.assert_allclose(fp @ u, 1.0, atol=1e-12)
        pm = V[r["free"][n, 1]]
        um = (pts[0] - pm) - np.dot(pts[0] - pm, (b - a)) / np.dot(b - a, b - a) * (b - a)
        um /= np.linalg.norm(um)
        np.testing.assert_allclose(fm @ (-um), 1.0, atol=1e-12)
        # total divergence: (+l/A+) A+ + (-l/A-) A- = 0, and f is tangent on each side
        tp, tm = r["tri"][n]
        assert abs(r["length"][n] / r["area"][tp] * r["area"][tp] - r["length"][n] / r["area"][tm] * r["area"][tm]) < 1e-15


def test_mesh_errors():
    V, F = workloads.plate(2, 2, 1.0)
    F3 = np.concatenate([F, F[:1]], axis=0)           # a third triangle on the same edges
    with pytest.raises(MeshError):
        build_rwg(V, F3)
    V2 = V.copy()
    V2[F[0, 1]] = V2[F[0, 0]]                          # collapse a triangle
    with pytest.raises(MeshError):
        build_rwg(V2, F)
    V3 = V.copy()
    V3[0, 0] = np.nan
    with pytest.raises(MeshError):
        build_rwg(V3, F)


# ---------------------------------------------------------------- potentials
def _brute_potentials(r, tv):
    """Adaptive polar quadrature about the projection of r (signed sub-triangles)."""
    n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
    n /= np.linalg.norm(n)
    d = np.dot(r - tv[0], n)
    rho = r - d * n
    e1 = (tv[1] - tv[0]) / np.linalg.norm(tv[1] - tv[0])
    e2 = np.cross(n, e1)
    I1 = 0.0
    Iv = np.zeros(3)
    for i in range(3):
        a, b = tv[i] - rho, tv[(i + 1) % 3] - rho
        pa = np.array([a @ e1, a @ e2])
        pb = np.array([b @ e1, b @ e2])
        area2 = pa[0] * pb[1] - pa[1] * pb[0]
        if abs(area2) < 1e-300:
            continue
        sgn = np.sign(area2)
        ta, tb = np.arctan2(pa[1], pa[0]), np.arctan2(pb[1], pb[0])
        dt = (tb - ta + np.pi) % (2 * np.pi) - np.pi
        # line through pa, pb: distance along direction theta
        nrm = np.array([pb[1] - pa[1], pa[0] - pb[0]])
        c = nrm @ pa

        def rmax(th):
            return c / (nrm @ np.array([np.cos(th), np.sin(th)]))

        def f0(th):
            return integrate.quad(lambda s: s / np.sqrt(s * s + d * d), 0, rmax(th), epsabs=1e-15, epsrel=1e-13)[0]

        def fv(th, comp):
            g = integrate.quad(lambda s: s * s / np.sqrt(s * s + d * d), 0, rmax(th), epsabs=1e-15, epsrel=1e-13)[0]
            return g * (np.cos(th) if comp == 0 else np.sin(th))

        th0, th1 = ta, ta + dt
        I1 += np.sign(dt) * sgn * sgn * integrate.quad(f0, min(th0, th1), max(th0, th1), epsabs=1e-14, epsrel=1e-12)[0]
        vx = np.sign(dt) * integrate.quad(fv, min(th0, th1), max(th0, th1), args=(0,), epsabs=1e-14, epsrel=1e-12)[0]
        vy = np.sign(dt) * integrate.quad(fv, min(th0, th1), max(th0, th1), args=(1,), epsabs=1e-14, epsrel=1e-12)[0]
        Iv += vx * e1 + vy * e2
    return I1, Iv


@pytest.mark.parametrize("where", ["inside_onplane", "inside_offplane", "outside_onplane",
                                   "outside_offplane", "near_edge", "above_vertex"])
def test_potential_integrals_vs_adaptive(where):
    tv = np.array([[0.1, -0.2, 0.3], [1.2, 0.1, 0.5], [0.3, 0.9, 0.1]])
    n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
    n /= np.linalg.norm(n)
    c = tv.mean(0)
    r = {"inside_onplane": c + 0.1 * (tv[0] - c),
         "inside_offplane": c + 0.3 * n,
         "outside_onplane": tv[1] + 0.7 * (tv[1] - c),
         "outside_offplane": tv[2] + 0.4 * (tv[2] - c) - 0.25 * n,
         "near_edge": 0.5 * (tv[0] + tv[1]) + 1e-3 * (c - 0.5 * (tv[0] + tv[1])) + 1e-4 * n,
         "above_vertex": tv[0] + 0.05 * n}[where]
    I1, Iv = potential_integrals(r[None], tv[None])
    J1, Jv = _brute_potentials(r, tv)
    assert abs(I1[0] - J1) < 1e-10 * abs(J1)
    assert np.linalg.norm(Iv[0] - Jv) < 1e-9 * np.linalg.norm(Jv)


# ---------------------------------------------------------------- Z
def test_Z_symmetric_and_rows(sphere_small):
    V, F, Z, _ = sphere_small
    assert np.abs(Z - Z.T).max() < 1e-13 * np.abs(Z).max()
    rows = efie.rows_Z(V, F, K0, [0, 17, 301])
    assert np.abs(rows - Z[[0, 17, 301]]).max() < 1e-12 * np.abs(Z).max()


def test_R_psd_and_equals_planewave_form(sphere_small):
    V, F, Z, _ = sphere_small
    R = Z.real
    R6, R6i = planewave.R_planewave(V, F, K0)
    ev6 = np.linalg.eigvalsh(R6)
    assert ev6.min() > -1e-13 * ev6.max()          # exactly PSD by construction
    ev = np.linalg.eigvalsh(R)
    assert ev.min() > -1e-8 * ev.max()              # mixed form: quadrature error of the integration by parts
    assert ev.max() > 0
    # a wrong sign of R, a dropped divergence term or a wrong prefactor all fail this
    assert np.linalg.norm(R - R6) < 1e-6 * np.linalg.norm(R6)
    assert np.abs(R6i).max() < 1e-12 * np.abs(R6).max()


def test_dZdk_matches_central_difference(sphere_small):
    V, F, Z, dZ = sphere_small
    h = 1e-4 * K0
    Zp = efie.dense_Z(V, F, K0 + h)
    Zm = efie.dense_Z(V, F, K0 - h)
    fd = (Zp - Zm) / (2 * h)
    assert np.linalg.norm(dZ - fd) < 1e-7 * np.linalg.norm(dZ)


# ---------------------------------------------------------------- characteristic values
def _golden_table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_sphere.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()[1:]])
    return np.array(rows)


def test_closed_form_reproduces_table2():
    tab = _golden_table2()
    x = 1.5 * np.pi
    tm1 = modes.sphere_cv(1, x, "TM")
    te3 = modes.sphere_cv(3, x, "TE")
    assert tm1 < 0 < te3                            # signs of Table II
    # finest mesh (15,015 unknowns) within its discretisation error of the closed form
    assert np.all(np.abs(tab[:3, 4] - tm1) < 3.0e-3)
    assert np.all(np.abs(tab[3:, 4] - te3) < 2.0e-3)
    # and the error shrinks with refinement across the three meshes
    e = np.abs(tab[:3, [2, 3, 4]] - tm1).mean(axis=0)
    assert e[0] > e[1] > e[2]
    # the smallest closed-form values at ka = 1.5 pi are TM1 (x3) then TE3 (x7)
    sm = modes.sphere_smallest(x, 10)
    np.testing.assert_allclose(sm[:3], tm1)
    np.testing.assert_allclose(sm[3:10], te3)


def test_closed_form_derivatives_match_finite_difference():
    a = 0.5
    for kind in ("TE", "TM"):
        for n in (1, 2, 3):
            h = 1e-6
            fd = (modes.sphere_cv(n, (K0 + h) * a, kind) - modes.sphere_cv(n, (K0 - h) * a, kind)) / (2 * h)
            assert abs(modes.sphere_dcv_dk(n, K0, a, kind) - fd) < 1e-6 * max(1, abs(fd))
    assert abs(modes.sphere_dcv_dk(1, K0, 0.5, "TE") + 0.5) < 1e-12


def test_qz_sphere_converges_to_closed_form(sphere_small, sphere_cfg1):
    x = np.pi
    exact = np.sort(modes.sphere_smallest(x, 10))   # TM3 (2 of 7), TE1 x3, TE2 x5
    errs = []
    for _, _, Z, *rest in (sphere_small, sphere_cfg1):
        lam = modes.qz_modes(Z.imag, Z.real, nev=10)
        assert np.abs(lam.imag).max() < 1e-8
        lam = np.sort(lam.real)
        errs.append(np.abs(lam - exact).max())
        # degeneracy of the clusters is reproduced
        assert np.ptp(lam[2:5]) < 1e-6 and np.ptp(lam[5:]) < 1e-6
    assert errs[1] < 0.012
    assert errs[0] / errs[1] > 3.0                   # O(h^2) convergence


@pytest.mark.slow
def test_qz_sphere_r075_between_table2_columns():
    """Icosphere nsub 3 at radius 0.75 wavelength: 1,920 unknowns, between the
    paper's 942- and 3,519-unknown meshes, so its values must fall between the
    two MoM+QZ columns of Table II."""
    tab = _golden_table2()
    V, F = workloads.icosphere(3, 0.75)
    Z = efie.dense_Z(V, F, K0)
    lam = np.sort(modes.qz_modes(Z.imag, Z.real, nev=8).real)
    lo = np.minimum(tab[:, 0], tab[:, 1])
    hi = np.maximum(tab[:, 0], tab[:, 1])
    assert np.all(lam[:3] > lo[:3].min() - 1e-3) and np.all(lam[:3] < hi[:3].max() + 1e-3)
    assert np.all(lam[3:] > lo[3:].min() - 1e-3) and np.all(lam[3:] < hi[3:].max() + 1e-3)


def test_dlambda_dk_oracle_vs_qz_difference_and_closed_form(sphere_small):
    V, F, Z, dZ = sphere_small
    lam, J = modes.qz_modes(Z.imag, Z.real, nev=3, vectors=True)
    lam = lam.real
    d = modes.dlambda_dk_cluster(J, lam, dZ.imag, dZ.real, Z.real)
    h = 1e-4 * K0
    lp = np.sort(modes.qz_modes(efie.dense_Z(V, F, K0 + h).imag, efie.dense_Z(V, F, K0 + h).real, nev=3).real)
    lm = np.sort(modes.qz_modes(efie.dense_Z(V, F, K0 - h).imag, efie.dense_Z(V, F, K0 - h).real, nev=3).real)
    fd = (lp - lm) / (2 * h)
    np.testing.assert_allclose(np.sort(d), np.sort(fd), rtol=1e-5, atol=1e-7)
    # same order of magnitude as the closed form (mesh nsub 2 is coarse)
    assert abs(np.mean(d) - modes.sphere_dcv_dk(1, K0, 0.5, "TE")) < 0.1


# ---------------------------------------------------------------- translators (point test)
@pytest.mark.parametrize("a", [0.25, 0.5, 1.0, 2.0])
def test_sin_expansion_accurate_in_both_cases(a):
    for case in (1, 2):
        err, rhs, lhs = translators.point_test("j", case, a)
        assert err < 1e-6
        assert abs(rhs.imag) < 1e-8 * abs(rhs.real)   # spurious imaginary part negligible


def test_cos_and_full_expansion_behaviour():
    # case 1 (addition theorem valid): error falls with box size
    e = [translators.point_test("y", 1, a)[0] for a in (0.25, 1.0, 2.0)]
    assert e[2] < e[1] < e[0] and e[2] < 1e-4
    eh = [translators.point_test("h", 1, a)[0] for a in (0.25, 1.0, 2.0)]
    assert eh[2] < eh[1] < eh[0] and eh[2] < 1e-4
    # case 2 (theorem violated): cos fails
    assert translators.point_test("y", 2, 0.5)[0] > 0.5
    # more digits -> smaller error
    assert translators.point_test("h", 1, 0.5, d0=5)[0] < 0.5 * translators.point_test("h", 1, 0.5, d0=3)[0]


def test_truncation_rule():
    # eq. (30) with d0 = 3 at a quarter-wavelength box
    assert translators.truncation_L(K0, 0.25, 3.0) == 8
    assert translators.truncation_L(K0, 4.0, 3.0) == 57


def _subdivide(tv, n):
    tris = [tv]
    for _ in range(n):
        new = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            new += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = new
    return np.array(tris)


@pytest.mark.parametrize("shared", [2, 1, 0])
def test_near_singular_pair_vs_subdivided_quadrature(shared):
    """A near-singular pair of distinct (non-coplanar) triangles: the outer
    7-point rule with the extracted inner integral must match the same outer
    rule with a brute-force inner integral on 4^6 sub-triangles (the inner
    integrand is non-singular because the outer points are off the inner
    triangle).  Catches errors in the out-of-plane terms of the extraction."""
    V, F = workloads.icosphere(3, 0.5)
    geo = efie.Geometry(V, F)
    To = 0
    cand = np.flatnonzero(efie.near_singular(geo, np.zeros(F.shape[0], dtype=int), np.arange(F.shape[0])))
    nshare = np.array([len(set(F[To]) & set(F[t])) for t in cand])
    Ts = int(cand[np.flatnonzero(nshare == shared)[0]])      # shares an edge / a vertex / nothing
    assert efie.near_singular(geo, np.array([To]), np.array([Ts]))[0]
    S0, Sv, _ = efie.pair_blocks(K0, geo, np.array([To]), np.array([Ts]))
    sub = _subdivide(geo.tv[Ts], 6)
    pts = np.einsum("qa,tax->tqx", BARY, sub).reshape(-1, 3)
    ar = 0.5 * np.linalg.norm(np.cross(sub[:, 1] - sub[:, 0], sub[:, 2] - sub[:, 0]), axis=1)
    wts = (ar[:, None] * WEIGHTS[None, :]).ravel()
    for a in range(3):
        for b in range(3):
            acc0, accv = 0.0, 0.0
            for p in range(7):
                r = BARY[p] @ geo.tv[To]
                R = np.linalg.norm(r - pts, axis=1)
                g = wts * np.exp(-1j * K0 * R) / R
                acc0 += WEIGHTS[p] * geo.area[To] * np.sum(g)
                accv += WEIGHTS[p] * geo.area[To] * np.sum(g * ((pts - geo.tv[Ts][b]) @ (r - geo.tv[To][a])))
            assert abs(Sv[0, a, b] - accv) < 1e-4 * abs(accv)
        assert abs(S0[0] - acc0) < 1e-4 * abs(acc0)


def test_track_by_correlation_recovers_a_shuffle():
    """Modes at the 'next' wavenumber = a shuffled, sign-flipped, slightly
    perturbed copy of the current ones: the brute-force correspondence finds
    the shuffle, with correlations near 1."""
    rng = np.random.default_rng(11)
    n, m = 40, 5
    A = rng.standard_normal((n, n))
    R = A @ A.T + n * np.eye(n)
    J = rng.standard_normal((n, m))
    perm = np.array([3, 0, 4, 1, 2])
    Jb = np.empty_like(J)
    Jb[:, perm] = J * np.array([1, -1, 1, -1, 1])[None, :]
    Jb += 0.02 * rng.standard_normal(Jb.shape)
    p, c = modes.track_by_correlation(J, Jb, R)
    np.testing.assert_array_equal(p, perm)
    assert c.min() > 0.95
    C = modes.modal_correlation(J, J, R)
    np.testing.assert_allclose(np.diag(C), 1.0, rtol=1e-12)


def test_plate_mode_tracking_agrees_with_dlambda_dk():
    """A 1.0 m x 0.6 m plate (the paper's sweep geometry, coarse mesh) at 300
    and 305 MHz: the modes matched by correlation are the ones the first-order
    prediction lambda + (d lambda/dk) dk points to, even with the second
    frequency's modes shuffled; the prediction error is second order."""
    c0 = 299792458.0
    V, F = workloads.plate(10, 6, 0.1)
    k1, k2 = 2 * np.pi * 300e6 / c0, 2 * np.pi * 305e6 / c0
    Z1, dZ1 = efie.dense_Z(V, F, k1, deriv=True)
    Z2 = efie.dense_Z(V, F, k2)
    l1, J1 = modes.qz_modes(Z1.imag, Z1.real, nev=4, vectors=True)
    l2, J2 = modes.qz_modes(Z2.imag, Z2.real, nev=6, vectors=True)
    l1, l2 = l1.real, l2.real
    shuffle = np.array([4, 2, 0, 5, 1, 3])
    l2s, J2s = l2[shuffle], J2[:, shuffle]
    p, c = modes.track_by_correlation(J1, J2s, Z2.real)
    d = modes.dlambda_dk(J1, l1, dZ1.imag, dZ1.real, Z1.real)
    pred = l1 + d * (k2 - k1)
    print("lambda(300 MHz)", l1, "predicted", pred, "tracked", l2s[p], "corr", c)
    assert c.min() > 0.9
    nearest = np.array([np.argmin(np.abs(l2s - q)) for q in pred])
    np.testing.assert_array_equal(p, nearest)
    step = np.abs(d * (k2 - k1))
    err = np.abs(l2s[p] - pred)
    assert np.all(err < 0.15 * step)
    # second order: at half the step the prediction error drops about 4x
    kh = 0.5 * (k1 + k2)
    Zh = efie.dense_Z(V, F, kh)
    lh, Jh = modes.qz_modes(Zh.imag, Zh.real, nev=6, vectors=True)
    ph, ch = modes.track_by_correlation(J1, Jh, Zh.real)
    errh = np.abs(lh.real[ph] - (l1 + d * (kh - k1)))
    print("prediction error, full / half step", err, errh)
    assert ch.min() > 0.9
    assert np.all(errh < 0.35 * err)
