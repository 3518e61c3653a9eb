"""Seeded synthetic problem definitions for the time-space fractional
convection-diffusion equation (TSFCDE), problem (1.1) of Gu, Huang, Ji,
Carpentieri and Alikhanov, arXiv:1603.00279.

This package only *describes problems*: coefficient functions, initial data,
closed-form manufactured solutions and the source terms they imply, and the
seeded parameter draws of the benchmark workloads.  It contains none of the
difference scheme's arithmetic: no grid, no sampling instants, no weights,
no time-discretisation tables, no matrices, no solver.  Both the CPU oracle and the GPU path take their inputs
from here; neither imports the other.
"""
from .problems import (  # noqa: F401
    Problem,
    ManufacturedSolution,
    example1,
    example2,
    config_small,
    config_large,
    config_large_constant,
    batched_instances,
    warmstart_instances,
    HELD_OUT,
    SEED_BASE,
    device_sources,
    Problem2D,
    problem_2d,
    device_sources_2d,
    Problem3D,
    problem_3d,
    device_sources_3d,
)
