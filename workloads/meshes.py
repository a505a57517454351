"""Deterministic triangle meshes (vertices float64, faces int32, CCW seen from
outside / from +z).

* icosphere: a regular icosahedron whose faces are split into four by edge
  midpoints ``nsub`` times, every vertex projected onto the sphere of the given
  radius.  nsub = 3, 6, 8 give 1,280 / 81,920 / 1,310,720 triangles.
* plate: a square or rectangular grid in the plane z = 0, each cell split into
  two triangles by the diagonal from its lower-left to its upper-right corner.
"""
import numpy as np

_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array([(-1, _T, 0), (1, _T, 0), (-1, -_T, 0), (1, -_T, 0),
                   (0, -1, _T), (0, 1, _T), (0, -1, -_T), (0, 1, -_T),
                   (_T, 0, -1), (_T, 0, 1), (-_T, 0, -1), (-_T, 0, 1)], dtype=np.float64)
_ICO_F = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
                   (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
                   (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
                   (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], dtype=np.int64)


def icosphere(nsub: int, radius: float):
    """Return (V, F) of an icosahedral sphere mesh with 20*4**nsub triangles."""
    V = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    F = _ICO_F.copy()
    for _ in range(nsub):
        nv = V.shape[0]
        # unique undirected edges, numbered in order of first appearance
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        key = np.sort(e, axis=1)
        code = key[:, 0] * (nv + 1) + key[:, 1]
        uniq, first, inv = np.unique(code, return_index=True, return_inverse=True)
        order = np.argsort(first, kind="stable")          # first-appearance order
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        mid_id = nv + rank[inv]
        ukey = key[first[order]]
        M = 0.5 * (V[ukey[:, 0]] + V[ukey[:, 1]])
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        V = np.concatenate([V, M], axis=0)
        nf = F.shape[0]
        ab, bc, ca = mid_id[:nf], mid_id[nf:2 * nf], mid_id[2 * nf:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.stack([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
                      np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)], axis=1).reshape(-1, 3)
    return np.ascontiguousarray(V * float(radius)), np.ascontiguousarray(F.astype(np.int32))


def plate(nx: int, ny: int, h: float):
    """Return (V, F) of an nx-by-ny cell plate of spacing h centred at the origin, z = 0."""
    xs = (np.arange(nx + 1) - nx / 2.0) * h
    ys = (np.arange(ny + 1) - ny / 2.0) * h
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)

    def vid(i, j):
        return i * (ny + 1) + j

    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    i, j = i.ravel(), j.ravel()
    t1 = np.stack([vid(i, j), vid(i + 1, j), vid(i + 1, j + 1)], 1)
    t2 = np.stack([vid(i, j), vid(i + 1, j + 1), vid(i, j + 1)], 1)
    F = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return np.ascontiguousarray(V), np.ascontiguousarray(F.astype(np.int32))
