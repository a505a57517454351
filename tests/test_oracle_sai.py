"""Pins of the SAI oracle (parity unpinned by the paper: its thresholds are
undefined there; these pin the least-squares construction itself)."""
import numpy as np

from oracle.sai import sai


def test_block_diagonal_gives_exact_inverse():
    # well-separated diagonal blocks whose entries all pass the thresholds:
    # every column's LS problem is square and consistent, so P = Z^-1
    rng = np.random.default_rng(5)
    blocks = []
    for n in (3, 5, 4):
        B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
        blocks.append(B)
    N = sum(b.shape[0] for b in blocks)
    Z = np.zeros((N, N), dtype=complex)
    o = 0
    for B in blocks:
        Z[o:o + B.shape[0], o:o + B.shape[0]] = B
        o += B.shape[0]
    P = sai(Z, 1e-8, 1e-8, 0.0)
    np.testing.assert_allclose(P, np.linalg.inv(Z), atol=1e-12)


def test_single_entry_pattern_closed_form():
    # pattern {j} only: p = conj(a_j) / ||a||^2 with a = column j of Z~
    rng = np.random.default_rng(6)
    N = 12
    Z = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Z = Z + Z.T + 10 * np.eye(N)
    P = sai(Z, 0.0, 1.0, 0.0)            # eps2 = 1: only entries at least as large as the diagonal
    for j in range(N):
        col = Z[:, j]
        J = np.flatnonzero(np.abs(col) >= np.abs(Z[j, j]))
        if list(J) == [j]:
            a = col                       # Z~ = Z for eps1 = 0
            np.testing.assert_allclose(P[j, j], np.conj(a[j]) / np.vdot(a, a), rtol=1e-12)


def test_residual_orthogonal_to_pattern_columns():
    # normal equations of each column's LS problem hold
    rng = np.random.default_rng(7)
    N = 40
    Z = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Z[np.abs(Z) < 1.0] = 0
    Z = Z + Z.T + 6 * np.eye(N)
    P = sai(Z, 0.05, 0.3, 0.0)
    d = np.abs(np.diag(Z))
    Zt = np.where(np.abs(Z) >= 0.05 * d[None, :], Z, 0)
    for j in range(N):
        J = np.flatnonzero((np.abs(Z[:, j]) >= 0.3 * d[j]) & (Z[:, j] != 0))
        r = np.eye(N)[:, j] - Zt[:, J] @ P[J, j]
        assert np.abs(Zt[:, J].conj().T @ r).max() < 1e-12


def _near_count_by_box_histogram(V, F, nlv):
    """Number of near pairs counted a second way: RWG functions binned into
    leaf boxes (edge midpoint, floor), then sum over pairs of boxes at
    Chebyshev distance <= 1 of the product of their populations."""
    from collections import Counter
    from oracle.rwg import build_rwg
    V = np.asarray(V, dtype=np.float64)
    r = build_rwg(V, F)
    mid = 0.5 * (V[r["edge"][:, 0]] + V[r["edge"][:, 1]])
    lo, hi = V.min(0), V.max(0)
    side = (hi - lo).max() * (1 + 1e-9)
    n = 2 ** (nlv - 1)
    a = side / n
    origin = 0.5 * (lo + hi) - 0.5 * side
    boxes = Counter()
    for p in mid:
        boxes[tuple(min(n - 1, max(0, int(np.floor(c)))) for c in (p - origin) / a)] += 1
    total = 0
    for (i, j, k), cnt in boxes.items():
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    total += cnt * boxes.get((i + di, j + dj, k + dk), 0)
    return total


def test_near_mask_counts():
    """near_mask against an independent count by box populations, on the
    1,920-unknown sphere (3 levels) and a small plate lying on the octree's
    mid-plane (4 levels), and the survey's count of 846,744 near pairs for
    the sphere; symmetric with a full diagonal."""
    import workloads
    from oracle.sai import near_mask
    V, F = workloads.icosphere(3, 0.5)
    m = near_mask(V, F, 3)
    assert m.sum() == 846744
    assert m.sum() == _near_count_by_box_histogram(V, F, 3)
    assert np.array_equal(m, m.T) and m.diagonal().all()
    V, F = workloads.plate(12, 10, 0.1)
    m = near_mask(V, F, 4)
    assert m.sum() == _near_count_by_box_histogram(V, F, 4)
    assert np.array_equal(m, m.T) and m.diagonal().all()


def test_near_count_plate_10x10():
    """The 10 x 10 wavelength plate (29,800 unknowns, 6 levels): the near
    pairs by box populations agree with the survey's independent count of
    7.52M (7,520,170 here)."""
    import workloads
    V, F, spec = workloads.workload("plate_10x10_n29800")
    c = _near_count_by_box_histogram(V, F, spec["nlv"])
    print("plate near pairs", c)
    assert abs(c - 7.52e6) < 0.005e6
