"""Seeded standard complex normal vectors CN(0, 1): real and imaginary parts
independent N(0, 1/2), so E|z|^2 = 1.  numpy's PCG64 generator."""
import numpy as np


def cn01(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im) * np.sqrt(0.5)


def cn01_block(n: int, ncols: int, seed0: int) -> np.ndarray:
    """(n, ncols) complex128 block; column j is cn01(n, seed0 + j)."""
    out = np.empty((n, ncols), dtype=np.complex128)
    for j in range(ncols):
        out[:, j] = cn01(n, seed0 + j)
    return out
