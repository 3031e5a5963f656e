"""SRJ (Scheduled Relaxation Jacobi) Poisson solver for AMD Instinct MI355X (gfx950).

The solver is the HIP library ``libsrj.so`` (C ABI in ``include/srj.h``); ``srj`` is its
ctypes binding and ``autograd`` wraps it as a differentiable PyTorch function.
``workloads`` draws the seeded synthetic inputs.
"""
from .srj import (SrjError, srj_plan, srj_plan_describe, srj_plan_sequence,  # noqa: F401
                  srj_plan_set_fusion, srj_residual, srj_schedule_optimal, srj_schedule_order,
                  srj_solve, srj_solve_ir, srj_sweeps)
