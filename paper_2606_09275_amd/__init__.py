"""MI355X (gfx950) implementation of the per-Newton-iteration assembly of the implicit
octree-based adaptive GIMP material point method: octree with hanging-node constraints,
Morton-ordered points, fused basis/kinematics/Hencky-von Mises/tangent kernel with per-leaf
LDS reduction, FP64 and FP32-tangent variants, and the adjoint assembly.

The compute path is the HIP library libmpmgimp.so behind the C ABI of include/mpm_gimp.h;
this package only marshals torch tensors to it. Importing the package does not load the
library; the first call does, and raises if it has not been built."""
from ._lib import MPM_F32K, MPM_F64, MPMError  # noqa: F401


def __getattr__(name):
    if name == "Mesh":
        from .mesh import Mesh
        return Mesh
    if name == "MPMForce":
        from .autograd import MPMForce
        return MPMForce
    raise AttributeError(name)
