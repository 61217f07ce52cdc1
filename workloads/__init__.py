"""Seeded synthetic inputs for the coupled lattice-Boltzmann / atom workloads.

This package builds initial conditions only (atom positions, velocities, bond lists,
body-force fields, loss targets, atom charges). It holds none of the method's arithmetic, so both the
CPU oracle and the HIP path consume the very same arrays.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    Workload,
    ball_atoms,
    confined_saw,
    globule_workload,
    make_workload,
    seeded_charges,
    small_workload,
)
