"""CPU FP64 oracle for the ACOPF model evaluation.

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the CPU
baseline leg of the benchmark.  The HIP path never imports it.
"""
from .acopf_oracle import (  # noqa: F401
    Model, branch_admittances, constraint_scales, constraints, evaluate,
    hessian_matrix, jacobian_matrix, jacobian_row_scales, objective, pattern, prepare, scales, vjp,
    vjp_scale,
)
