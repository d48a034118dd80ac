"""Test oracle: a plain, slow, FP64 scalar-CSR smoothed-aggregation AMG + CG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library: it reads the
inputs (scalar CSR matrix, node coordinates, right-hand side) and computes,
in scalar arithmetic throughout, what the paper's method computes:

* Algorithm 1 (setup): rigid body modes from coordinates, aggregation on the
  node strength graph, tentative prolongation by per-aggregate QR of the
  near-nullspace, Jacobi-smoothed prolongation, R = P^T, Galerkin A_{i+1} =
  R_i A_i P_i, smoother data, dense Cholesky of the coarsest matrix;
* Algorithm 2 (V-cycle), used as the preconditioner of conjugate gradients
  with a relative residual target (Section 4 uses 1e-8).

Where the paper is silent (the aggregation rule, strength threshold, damping
factors, smoother), the documented readings in ``oracle.setup`` apply.

Parity status per function is stated in each module's header.
"""
from .formats import csr_to_bsr, bsr_to_csr
from .nullspace import rigid_body_modes
from .setup import (AmgParams, Level, Hierarchy, build_hierarchy, strength_graph,
                    aggregate, tentative_prolongation, smoothed_prolongation,
                    jacobi_smoother, spai0_smoother, power_lambda_max)
from .solve import vcycle, pcg, amg_pcg, true_residual_norm, SolveResult

__all__ = [
    "csr_to_bsr", "bsr_to_csr", "rigid_body_modes", "AmgParams", "Level", "Hierarchy",
    "build_hierarchy", "strength_graph", "aggregate", "tentative_prolongation",
    "smoothed_prolongation", "jacobi_smoother", "spai0_smoother", "power_lambda_max", "vcycle", "pcg",
    "true_residual_norm", "SolveResult", "amg_pcg",
]
