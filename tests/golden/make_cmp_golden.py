"""Writes cmp_sphere_n1920.npz: the oracle's Calderon-preconditioner products
on the sphere of radius 0.5 wavelength meshed by the icosahedron subdivided
three times (1,280 triangles, 1,920 RWG; its barycentric refinement has
7,680 triangles and 11,520 RWG), at k = 2 pi, for the GPU parity tests:

  x    = cn01(1920, 7)                   (seeded input)
  Gx   = G x                             (mixed Gram matrix, eq. (27))
  rows = 64 BC rows (seed 5, without replacement)
  Ztx  = (Z~ x)[rows]                    (EFIE between BC functions, eq. (26))
  u    = G^-1 Z x
  Mx   = (Z~ G^-1 Z x)[rows]             (the matrix of eq. (25))
  b    = cn01(1920, 8), xs = Z^-1 b      (dense solve)
  lam  = the 8 characteristic values of smallest |lambda| (dense QZ)

Only oracle/ and the seeded input generators are used; the rows of Z~ are
split over `workers` processes (default 8; a few minutes in all):

    python tests/golden/make_cmp_golden.py [workers]
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads                      # noqa: E402
from oracle import cmp, efie, modes   # noqa: E402

K = 2 * np.pi


def _mesh():
    return workloads.icosphere(3, 0.5)


def _rows_job(args):
    rows, X = args
    os.environ["OMP_NUM_THREADS"] = "1"
    V, F = _mesh()
    return cmp.ztilde_rows(V, F, K, rows, X)


def main(workers=8):
    V, F = _mesh()
    Z = efie.dense_Z(V, F, K)
    N = Z.shape[0]
    B, Vr, Fr = cmp.bc_table(V, F)
    G = cmp.gram(V, F, B, Vr, Fr)
    x = workloads.cn01(N, 7)
    b = workloads.cn01(N, 8)
    rows = np.sort(np.random.default_rng(5).choice(N, 64, replace=False))
    X = np.stack([x, np.linalg.solve(G, Z @ x)], axis=1)       # Z~ of x and of G^-1 Z x
    parts = np.array_split(rows, workers)
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_rows_job, [(p, X) for p in parts])
    ZtX = np.concatenate(res, axis=0)
    lam = modes.qz_modes(Z.imag, Z.real, nev=8)
    out = dict(N=N, k=K, x=x, Gx=G @ x, rows=rows, Ztx=ZtX[:, 0], u=X[:, 1], Mx=ZtX[:, 1], b=b,
               xs=np.linalg.solve(Z, b),
               lam=np.asarray(lam))
    np.savez(os.path.join(HERE, "cmp_sphere_n1920.npz"), **out)
    print("wrote cmp_sphere_n1920.npz", N, np.round(np.sort(np.real(lam)), 6))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
