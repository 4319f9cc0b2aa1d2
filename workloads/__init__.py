"""Seeded synthetic junctions (wires) for the real-space NEGF transmission path.

This module only draws inputs: grid sizes, a local potential built from
Gaussian wells, Kleinman-Bylander (KB) projector values, per-plane complex
absorbing potential (CAP) profiles and energy grids.  It holds none of the
method's arithmetic (no finite differences, no Green's functions, no
transmission); both the CPU oracle and the GPU library consume its arrays.
"""

from .wires import (  # noqa: F401
    Wire,
    CONFIGS,
    make_wire,
    make_custom,
    make_junctions,
    rhs_columns,
    left_support,
    well_basis,
    potential_from_amplitudes,
    quartic_cap,
    power_cap,
    end_gaussian_cap,
    riss_meyer_cap,
    riss_meyer_error,
    riss_meyer_strength,
    with_caps,
)
