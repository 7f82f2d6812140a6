"""MI355X (gfx950) implementation of the implicit-Euler Projective Dynamics
step on hexahedral voxel meshes and its adjoint (DiffPD).

The simulation runs in libdiffpd.so (HIP kernels behind a C ABI, see
include/diffpd.h); this package only marshals arguments.
"""
from ._lib import load as load_library, DiffPDError  # noqa: F401

__all__ = ["load_library", "DiffPDError", "Mesh", "PDStep", "pd_step", "rollout"]


def __getattr__(name):
    if name == "Mesh":
        from .mesh import Mesh
        return Mesh
    if name in ("PDStep", "pd_step", "rollout"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
