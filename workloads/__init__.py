"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds input generation only: triangle meshes of the shapes the
paper analyses (PEC sphere, rectangular PEC plate) and seeded complex normal
vectors.  It contains none of the method's arithmetic (no basis functions, no
Green's function, no quadrature), so that the CPU oracle and the GPU library
can share inputs without sharing any computation.
"""
from .meshes import icosphere, plate
from .vectors import cn01, cn01_block
from .configs import WORKLOADS, workload

__all__ = ["icosphere", "plate", "cn01", "cn01_block", "WORKLOADS", "workload"]
