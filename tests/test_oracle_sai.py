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
