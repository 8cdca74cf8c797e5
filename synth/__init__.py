"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only *generates* inputs: triangle meshes of closed surfaces,
per-element pressure amplitudes and sampled load histories.  It holds none of
the boundary-element arithmetic (no normals, no kernels, no quadrature, no
transforms); each side of a parity test derives those on its own.
"""

from .mesh import icosphere, ellipsoid, merge_meshes, random_cavity_centres, box_mesh
from .loads import ramp_history, uniform_pressure, sh_pressure, ricker_history
from .configs import config_inputs, CONFIG_SEED_BASE

__all__ = [
    "icosphere", "ellipsoid", "merge_meshes", "random_cavity_centres", "box_mesh",
    "ramp_history", "uniform_pressure", "sh_pressure", "ricker_history",
    "config_inputs", "CONFIG_SEED_BASE",
]
