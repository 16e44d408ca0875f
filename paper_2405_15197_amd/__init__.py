"""latmesh: MI355X (gfx950) meta-meshing and triangulation of strut lattices.

The work is done by the HIP kernels in ``csrc/`` behind the C ABI of
``include/latmesh.h``; ``latmesh`` is its ctypes binding."""

from . import latmesh  # noqa: F401
from .latmesh import Mesher, MeshResult, LatmeshError  # noqa: F401
