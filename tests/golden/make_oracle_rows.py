"""Writes oracle_rows_<workload>.json: sampled rows of the oracle's Z (and of
its real and imaginary parts R and X) applied to the seeded test columns, for GPU parity tests at sizes where filling the
rows takes minutes (1,966,080 unknowns: about 40 s per row on one core).

Only oracle/ and the seeded input generators are used.  Rows: seed 2 (without
replacement); columns: the block of seeds 100 + j with column 0 replaced by
the seed-0 vector, the first `ncols` of them.

    python tests/golden/make_oracle_rows.py sphere_r12_n1966080 4 4
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads                      # noqa: E402
from oracle import efie               # noqa: E402
from oracle.rwg import build_rwg      # noqa: E402


def main(name, nrows, ncols):
    V, F, spec = workloads.workload(name)
    rwg = build_rwg(V, F)
    N = int(rwg["N"])
    rows = np.sort(np.random.default_rng(2).choice(N, nrows, replace=False))
    X = workloads.cn01_block(N, ncols, 100)
    X[:, 0] = workloads.cn01(N, 0)
    Zr = efie.rows_Z(V, F, spec["k"], rows, geo=efie.Geometry(V, F), rwg=rwg)
    Zx = Zr @ X
    Rx = Zr.real @ X          # R = Re Z, X = Im Z entry by entry (Z = R + iX)
    Xx = Zr.imag @ X
    out = {"workload": name, "N": N, "k": spec["k"], "rows": rows.tolist(), "ncols": ncols,
           "columns": "seeds 100 + j, column 0 = seed 0", "Zx_re": Zx.real.tolist(), "Zx_im": Zx.imag.tolist(),
           "Rx_re": Rx.real.tolist(), "Rx_im": Rx.imag.tolist(), "Xx_re": Xx.real.tolist(), "Xx_im": Xx.imag.tolist()}
    with open(os.path.join(HERE, f"oracle_rows_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]))
