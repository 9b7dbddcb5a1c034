"""Seeded synthetic inputs (Jacobians, right-hand sides) shared by tests and benchmark.

Holds no solver arithmetic: only the physics discretisation that produces inputs.
"""
from .jacobian import BSR, PoroSystem, build_system, make_rhs, q1_cube, two_phase, three_phase
from .configs import workload, serving_request, WORKLOADS

__all__ = ["BSR", "PoroSystem", "build_system", "make_rhs", "q1_cube", "two_phase",
           "three_phase", "workload", "serving_request", "WORKLOADS"]
