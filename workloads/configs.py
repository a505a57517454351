"""The five synthetic workloads (wavelength = 1, so k = 2*pi at the nominal
frequency).  Each entry names the mesh recipe and the tree depth (levels
counted from the root, level 0 included)."""
import math
from .meshes import icosphere, plate

WORKLOADS = {
    # PEC sphere radius 0.5 wavelength, 1,920 RWG unknowns, 3 levels
    "sphere_r0.5_n1920": dict(kind="sphere", nsub=3, radius=0.5, k=2 * math.pi, nlv=3),
    # PEC sphere radius 4 wavelengths, 122,880 RWG unknowns, 6 levels
    "sphere_r4_n122880": dict(kind="sphere", nsub=6, radius=4.0, k=2 * math.pi, nlv=6),
    # 10 x 10 wavelength plate, 0.1 wavelength cells, 29,800 RWG unknowns, 6 levels
    "plate_10x10_n29800": dict(kind="plate", nx=100, ny=100, h=0.1, k=2 * math.pi, nlv=6),
    # PEC sphere radius 12 wavelengths, 1,966,080 RWG unknowns, 8 levels
    "sphere_r12_n1966080": dict(kind="sphere", nsub=8, radius=12.0, k=2 * math.pi, nlv=8),
}


def workload(name: str):
    """Return (V, F, spec) for a named workload."""
    spec = dict(WORKLOADS[name])
    if spec["kind"] == "sphere":
        V, F = icosphere(spec["nsub"], spec["radius"])
    else:
        V, F = plate(spec["nx"], spec["ny"], spec["h"])
    return V, F, spec
