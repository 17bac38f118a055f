"""Seeded synthetic workload generators: grids, immersed bodies, initial fields,
case descriptions and the serving request stream.

This package is the only code shared by the HIP path and the CPU oracle.  It
holds none of the solver's arithmetic: it only produces coordinates,
connectivity, primitive initial fields and parameters.  Every coordinate it
emits is snapped to a dyadic lattice (faces to multiples of 2**-23, body
vertices to multiples of 2**-24) so that both implementations can take their
inside/outside decisions on exact integers.
"""
from .grids import (LATTICE_BITS, snap, uniform_faces, tanh_center_faces,
                    core_stretched_faces)
from .bodies import circle_polygon, wedge_polygon, naca00_polygon, star_polygon, tube_mesh, sphere_mesh
from .fields import freestream_prim, random_periodic_prim, entropy_wave_prim
from .cases import Case, case_c1, case_c2, case_c3, case_c4, small_case, CASES
from .serving import request_stream

__all__ = [
    "LATTICE_BITS", "snap", "uniform_faces", "tanh_center_faces",
    "core_stretched_faces", "circle_polygon", "wedge_polygon", "naca00_polygon", "star_polygon",
    "tube_mesh", "sphere_mesh", "freestream_prim", "random_periodic_prim", "entropy_wave_prim",
    "Case", "case_c1", "case_c2", "case_c3", "case_c4", "small_case", "CASES",
    "request_stream",
]
