"""Seeded synthetic inputs for the MetaDE inner-DE path.

This package generates problem instances (shifts, rotations, permutations,
linear systems) and workload descriptions (run sizes, streams, sampled
hyperparameter vectors).  It holds none of the method's arithmetic: no
sampling of DE indices, no mutation, crossover, fitness or selection.  Both
the CPU oracle and the GPU path read their inputs from here.
"""
from .synth import (  # noqa: F401
    KINDS, Problem, Workload, theta_box, make_rotation, make_problem,
    workload_c1, workload_c2, workload_c3, workload_c4, workload_c5, workload_paper,
    workload_t7, workload_c5e16, workload_by_name, small_batch, control_batch, mlp_param_count,
    TABLE7_HIDDEN, TABLE7_TASKS,
)
