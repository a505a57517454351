"""Writes oracle_rows_<workload>.npz: sampled rows of the oracle's Z (and of
its real and imaginary parts R and X) applied to the seeded test columns, for
GPU parity tests at sizes where filling the rows takes minutes or hours
(122,880 unknowns: about 1 s per row on one core; 1,966,080 unknowns: about
40 s per row).

Only oracle/ and the seeded input generators are used.  Rows: seed 2 (without
replacement); columns: the block of seeds 100 + j with column 0 replaced by
the seed-0 vector, the first `ncols` of them.  Rows are split over `workers`
processes (each fills its rows independently; the result does not depend on
the split).

    python tests/golden/make_oracle_rows.py sphere_r4_n122880 1229 32 8
    python tests/golden/make_oracle_rows.py sphere_r12_n1966080 256 8 4

The arrays (numpy .npz, no pickled objects): rows (int64), Zx, Rx, Xx
(len(rows) x ncols complex128), N, k, ncols.
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads                      # noqa: E402
from oracle import efie               # noqa: E402
from oracle.rwg import build_rwg      # noqa: E402

_G = {}


def _init(name, ncols):
    V, F, spec = workloads.workload(name)
    rwg = build_rwg(V, F)
    N = int(rwg["N"])
    X = workloads.cn01_block(N, ncols, 100)
    X[:, 0] = workloads.cn01(N, 0)
    _G.update(V=V, F=F, k=spec["k"], rwg=rwg, geo=efie.Geometry(V, F), X=X)


def _rows(chunk):
    g = _G
    out = []
    for m in chunk:
        Zr = efie.rows_Z(g["V"], g["F"], g["k"], np.array([m]), geo=g["geo"], rwg=g["rwg"])
        # R = Re Z and X = Im Z entry by entry (Z = R + iX)
        out.append((m, Zr @ g["X"], Zr.real @ g["X"], Zr.imag @ g["X"]))
    return out


def oracle_row_products(name, nrows, ncols, workers=1):
    """(rows, Zx, Rx, Xx, N, k) for the seeded rows and columns of `name`."""
    V, F, spec = workloads.workload(name)
    N = int(build_rwg(V, F)["N"])
    rows = np.sort(np.random.default_rng(2).choice(N, nrows, replace=False))
    chunks = [rows[i::max(1, 4 * workers)] for i in range(max(1, 4 * workers))]
    chunks = [c for c in chunks if c.size]
    res = {}
    t0 = time.time()
    if workers <= 1:
        _init(name, ncols)
        for c in chunks:
            for m, z, r, x in _rows(c):
                res[m] = (z, r, x)
    else:
        with mp.get_context("fork").Pool(workers, initializer=_init, initargs=(name, ncols)) as pool:
            for part in pool.imap_unordered(_rows, chunks):
                for m, z, r, x in part:
                    res[m] = (z, r, x)
                print(f"{len(res)}/{rows.size} rows ({time.time() - t0:.0f} s)", flush=True)
    Zx = np.concatenate([res[m][0] for m in rows], axis=0)
    Rx = np.concatenate([res[m][1] for m in rows], axis=0)
    Xx = np.concatenate([res[m][2] for m in rows], axis=0)
    return rows, Zx, Rx, Xx, N, spec["k"]


def main(name, nrows, ncols, workers):
    rows, Zx, Rx, Xx, N, k = oracle_row_products(name, nrows, ncols, workers)
    np.savez(os.path.join(HERE, f"oracle_rows_{name}.npz"), rows=rows.astype(np.int64), Zx=Zx, Rx=Rx, Xx=Xx,
             N=np.int64(N), k=np.float64(k), ncols=np.int64(ncols))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]) if len(sys.argv) > 4 else 1)
