"""Seeded synthetic 3D linear-elasticity problems (Q1 hexahedra and Kuhn-split
P1 tetrahedra, 3x3 node blocks).

This module builds the *inputs* of the solver: the stiffness matrix in block CSR
form with 3x3 blocks, the node coordinates and the right-hand sides.  It holds
none of the multigrid method's arithmetic (no rigid body modes, no aggregation,
no transfer operators, no smoothers) and is shared by the test oracle, the
tests and the benchmark as their single source of seeded inputs.
"""
from .elasticity import (
    Problem,
    q1_element_stiffness,
    assemble_box,
    bsr_to_csr,
    cube_c1,
    cube_lognormal,
    cube_inclusions,
    cube_multi_rhs,
    batch_cubes,
    beam,
    training_beams,
    named_problem,
)
from .tets import p1_element_stiffness, assemble_tets, tet_cube, rod_standin, hook_standin

__all__ = [
    "Problem", "q1_element_stiffness", "assemble_box", "bsr_to_csr", "cube_c1",
    "cube_lognormal", "cube_inclusions", "cube_multi_rhs", "batch_cubes", "beam",
    "training_beams", "named_problem", "p1_element_stiffness", "assemble_tets", "tet_cube",
    "rod_standin", "hook_standin",
]
