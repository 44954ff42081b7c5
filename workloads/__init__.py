"""Seeded synthetic inputs (coefficient fields, initial conditions, workload configs).

This package only draws random inputs. It holds none of the method's arithmetic (no stencil,
no factorization, no time stepping), so both the CPU oracle's tests and the GPU path can take
their inputs from it without sharing any of the method's code.
"""
from .gen import (  # noqa: F401
    Workload,
    bumps,
    cell_centres,
    grf_coefficient,
    iid_loguniform_cells,
    iid_uniform_nodes,
    node_coords,
    poisson_arrivals,
    serving_request,
    serving_requests,
    spectral_grf_coefficient,
    sine_mode,
    workload,
    WORKLOADS,
    load_config,
    config_names,
)
