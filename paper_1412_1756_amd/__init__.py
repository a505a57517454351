"""MI355X (gfx950) MLFMA for characteristic-mode analysis.

``Operator`` wraps one library handle: it builds the RWG discretisation,
octree, interaction lists and device tables from a triangle mesh and a
wavenumber, then applies Z, R, X, Z^H (and dZ/dk) and the SAI preconditioner
to complex torch tensors that live on the GPU.  Torch supplies device memory
and the stream; the arithmetic runs in the library's HIP kernels.
"""
from .operator import Operator, CmError

__all__ = ["Operator", "CmError"]
