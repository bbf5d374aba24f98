"""FP64 CPU oracle for the ETD2RKds hot path (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow, readable reference against which the HIP
path is checked.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2307_10684_amd``) never does, and this package never imports the
product path.  The two share no code: the only common module is ``synth``,
which draws seeded inputs and holds none of the method's arithmetic.

Every function follows a passage of Caliari & Cassini, "A second order
directional split exponential integrator for systems of
advection-diffusion-reaction equations" (arXiv 2307.10684), cited by section
and equation number.  Arithmetic is numpy float64 throughout; the only
library primitives used as steps are ``numpy.tensordot`` (the mu-mode product
as a matrix product on an unfolding) and ``numpy.kron`` (dense Kronecker
sums for tiny grids).

Parity status of each function is stated in its docstring; every function
has at least one pin in ``tests/test_oracle_*.py`` against mathematics or
printed values that do not come from the oracle itself.
"""
from .operators import (grid_nodes, laplacian_1d, advection_1d, operator_1d,
                        kron_sum_dense)
from .matfun import expm_taylor, phi_functions, phi_scalar
from .tensor import vec, unvec, mode_product, tucker, kron_sum_action
from .models import reaction
from .integrators import (Problem, problem_from_workload, precompute, etd2rkds_step,
                          lawson2b_step, etd2rk_dense_step, solve, split_phi_dense)
from .metrics import relative_error, observed_order, rel_inf_error
from .indicators import (trapezoid_weights, spatial_mean, increment_norm, nonfinite_count,
                         indicators)

__all__ = [
    "grid_nodes", "laplacian_1d", "advection_1d", "operator_1d", "kron_sum_dense",
    "expm_taylor", "phi_functions", "phi_scalar",
    "vec", "unvec", "mode_product", "tucker", "kron_sum_action",
    "reaction",
    "Problem", "problem_from_workload", "precompute", "etd2rkds_step",
    "lawson2b_step", "etd2rk_dense_step", "solve", "split_phi_dense",
    "relative_error", "observed_order", "rel_inf_error",
    "trapezoid_weights", "spatial_mean", "increment_norm", "nonfinite_count", "indicators",
]
