"""Seeded synthetic inputs for the CC-MSAV vesicle step.

This package only draws initial conditions and parameter sets. It holds none
of the scheme's arithmetic, so the oracle and the HIP path can both consume it
without sharing any of the method.
"""
from .generators import (  # noqa: F401
    DEFAULT_DT,
    VESICLE_DT,
    ENSEMBLE_DT,
    WORKLOADS,
    GENERAL_SETS,
    general_dt,
    general_member,
    general_params,
    Member,
    circle_member,
    vesicle_member,
    make_workload,
    table_g_params,
    vesicle_dt,
)
