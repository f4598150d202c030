"""Seeded synthetic specimens and inputs for STEM-EELS map simulations.

This package only *produces input arrays* (atom lists, projected potentials,
transition potentials, probe positions and the problem description).  It holds
none of the simulation method's arithmetic: both the CPU oracle and the HIP
library consume what it emits, and neither shares any other code.
"""
from .specimens import (  # noqa: F401
    Problem,
    config1,
    config2,
    config3,
    config3_subproblem,
    config4,
    config5_stream,
    random_lattice_specimen,
    specimen_pool,
    random_problem,
    tiled_problem,
    probe_grid,
    transitions_lm,
    thermal_displacement,
)
