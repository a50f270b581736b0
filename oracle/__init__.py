"""CPU oracle for the RICI pipeline -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its binding) never calls
it, and the two share no code.
"""

from .oracle import (  # noqa: F401
    NBINS,
    build,
    load,
    lib_path,
    rici_rowrange,
    rici_brute,
    project,
    crd,
    distance_matrix,
    rank,
    threads,
    spin_images,
    pearson,
    pearson_matrix,
    pearson_rank,
    clutter_areas,
    triangle_area_in_volume,
)
