"""Seeded synthetic scenes for the RICI pipeline.

This package only builds inputs: triangle meshes (fp32 positions, u32 triangle
indices), oriented points (fp32 positions and area-weighted normals) and the
true-match map used by the rank search.  It contains none of the descriptor or
distance arithmetic, so both the HIP path and the CPU oracle can consume its
arrays without sharing any of the method's code.
"""

from .meshes import (  # noqa: F401
    Mesh,
    icosphere,
    cube_sphere,
    superquadric,
    torus,
    vertex_normals,
    normalize_to_unit_sphere,
    random_rotation,
    transform,
    concat,
    sample_surface,
)
from .images import step_images, perturb  # noqa: F401
from .configs import (  # noqa: F401
    Scene,
    config1_icosphere,
    config2_union12,
    config3_clutter,
    config4_batch,
    config5_database,
    config5_request,
    CONFIG_BUILDERS,
)
