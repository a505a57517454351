"""Seven-point, degree-5 triangle quadrature (Radon's rule).

The paper's Galerkin integrals (eq. (5)) need a triangle rule it does not
name; this build fixes the classical 7-point rule, exact for every polynomial
of total degree <= 5.  Points are barycentric; weights sum to one and are
multiplied by the triangle area by the caller.
"""
import numpy as np

_S15 = np.sqrt(15.0)
_A = (6.0 - _S15) / 21.0
_B = (6.0 + _S15) / 21.0
_WA = (155.0 - _S15) / 1200.0
_WB = (155.0 + _S15) / 1200.0

BARY = np.array([
    [1 / 3, 1 / 3, 1 / 3],
    [_A, _A, 1 - 2 * _A], [_A, 1 - 2 * _A, _A], [1 - 2 * _A, _A, _A],
    [_B, _B, 1 - 2 * _B], [_B, 1 - 2 * _B, _B], [1 - 2 * _B, _B, _B],
])
WEIGHTS = np.array([9.0 / 40.0, _WA, _WA, _WA, _WB, _WB, _WB])


def tri_points(tv: np.ndarray) -> np.ndarray:
    """Quadrature points of triangles tv (..., 3 vertices, 3 xyz) -> (..., 7, 3)."""
    return np.einsum("qa,...ax->...qx", BARY, tv)
