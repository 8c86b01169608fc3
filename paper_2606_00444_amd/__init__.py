"""MI355X-native per-frame dynamic mesh-Gaussian update.

Python face of libmgu.so (C ABI in include/mgu.h; HIP kernels for gfx950 in
csrc/).  The library implements the runtime side of "Real-Time Physics
Simulation with Dynamic Mesh-Gaussian Reconstructions" (arXiv 2606.00444):
vertex-buffer updates of a fixed-topology physics mesh, Gaussians re-posed
from their faces, a BVH built once and refit per frame, closest-point queries
with on-demand normals, the rebuild-per-frame comparison path, and a
differentiable template projection.  PyTorch provides device memory and
streams only.  If libmgu.so has not been built, every call raises.
"""

from .api import *  # noqa: F401,F403
from .api import __all__ as _api_all
from ._lib import MguError, MG_PRIM_POINTS, MG_PRIM_TRIANGLES, LIB_PATH

__all__ = list(_api_all) + ["MguError", "MG_PRIM_POINTS", "MG_PRIM_TRIANGLES", "LIB_PATH"]
